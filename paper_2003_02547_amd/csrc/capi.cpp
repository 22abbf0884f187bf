// C-ABI of the batched OCP-QP IPM: caller-owned memory for every object,
// host-side packing into the padded device layout, launches per kernel
// variant on the caller's stream.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "../../include/oqp.h"
#include "internal.h"
#include "layout.h"

using oqp::DevStat;
using oqp::InstDesc;
using oqp::Layout;

static thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

extern "C" const char* oqp_last_error(void) { return g_err; }

// ---------------------------------------------------------------------------
// dims
// ---------------------------------------------------------------------------

extern "C" size_t oqp_dims_bytes(int N)
{
    if (N < 1) return 0;
    return align_up(sizeof(oqp_dims), 16) + align_up(6 * (size_t)(N + 1) * sizeof(int), 16);
}

extern "C" int oqp_dims_init(void* mem, size_t bytes, int N, oqp_dims** out)
{
    if (!mem || !out || N < 1) return fail(OQP_EINVAL, "oqp_dims_init: bad argument (N=%d)", N);
    if (bytes < oqp_dims_bytes(N)) return fail(OQP_ENOMEM, "oqp_dims_init: %zu bytes < %zu", bytes, oqp_dims_bytes(N));
    if ((uintptr_t)mem % 8) return fail(OQP_EINVAL, "oqp_dims_init: memory not 8-byte aligned");
    oqp_dims* d = (oqp_dims*)mem;
    int* a = (int*)((char*)mem + align_up(sizeof(oqp_dims), 16));
    std::memset(a, 0, 6 * (size_t)(N + 1) * sizeof(int));
    d->N = N;
    d->nx = a;
    d->nu = a + (N + 1);
    d->nbu = a + 2 * (N + 1);
    d->nbx = a + 3 * (N + 1);
    d->ng = a + 4 * (N + 1);
    d->ns = a + 5 * (N + 1);
    *out = d;
    return OQP_OK;
}

extern "C" int oqp_dims_set_soft(oqp_dims* d, int n, int ns)
{
    if (!d || n < 0 || n > d->N) return fail(OQP_EINVAL, "oqp_dims_set_soft: stage %d out of range", n);
    if (ns < 0 || ns > d->nbu[n] + d->nbx[n] + d->ng[n])
        return fail(OQP_EINVAL, "oqp_dims_set_soft: %d slacks at stage %d with %d constraint rows", ns, n,
                    d->nbu[n] + d->nbx[n] + d->ng[n]);
    d->ns[n] = ns;
    return OQP_OK;
}

bool dims_soft(const oqp_dims* d)
{
    for (int n = 0; n <= d->N; ++n)
        if (d->ns[n] > 0) return true;
    return false;
}

// slack counts that no longer fit the stage's rows (stage sizes set after them)
static int check_soft_dims(const oqp_dims* d, const char* who)
{
    for (int n = 0; n <= d->N; ++n)
        if (d->ns[n] > d->nbu[n] + d->nbx[n] + d->ng[n])
            return fail(OQP_EINVAL, "%s: %d slacks at stage %d exceed its %d constraint rows", who, d->ns[n], n,
                        d->nbu[n] + d->nbx[n] + d->ng[n]);
    return OQP_OK;
}

extern "C" int oqp_dims_set_stage(oqp_dims* d, int n, int nx, int nu, int nbu, int nbx, int ng)
{
    if (!d || n < 0 || n > d->N) return fail(OQP_EINVAL, "oqp_dims_set_stage: stage %d out of range", n);
    if (nx < 0 || nu < 0 || nbu < 0 || nbx < 0 || ng < 0 || nbu > nu || nbx > nx)
        return fail(OQP_EINVAL, "oqp_dims_set_stage: bad sizes at stage %d", n);
    d->nx[n] = nx;
    d->nu[n] = nu;
    d->nbu[n] = nbu;
    d->nbx[n] = nbx;
    d->ng[n] = ng;
    return OQP_OK;
}

// ---------------------------------------------------------------------------
// qp
// ---------------------------------------------------------------------------


static void stage_sizes(const oqp_dims* d, int n, size_t* sz)
{
    const int nx = d->nx[n], nu = d->nu[n], nxn = n < d->N ? d->nx[n + 1] : 0;
    const int nbu = d->nbu[n], nbx = d->nbx[n], ng = d->ng[n];
    sz[F_A] = (size_t)nxn * nx;
    sz[F_B] = (size_t)nxn * nu;
    sz[F_b] = nxn;
    sz[F_Q] = (size_t)nx * nx;
    sz[F_S] = (size_t)nu * nx;
    sz[F_R] = (size_t)nu * nu;
    sz[F_q] = nx;
    sz[F_r] = nu;
    sz[F_lbu] = sz[F_ubu] = nbu;
    sz[F_lbx] = sz[F_ubx] = nbx;
    sz[F_D] = (size_t)ng * nu;
    sz[F_C] = (size_t)ng * nx;
    sz[F_lg] = sz[F_ug] = ng;
    sz[F_Zl] = sz[F_Zu] = sz[F_zl] = sz[F_zu] = sz[F_lls] = sz[F_lus] = d->ns[n];
}

static void qp_offsets(const oqp_dims* dims, int64_t* doff, int64_t* ioff)
{
    int64_t od = 0, oi = 0;
    size_t sz[F_COUNT];
    for (int n = 0; n <= dims->N; ++n) {
        doff[n] = od;
        ioff[n] = oi;
        stage_sizes(dims, n, sz);
        for (int f = 0; f < F_COUNT; ++f) od += (int64_t)sz[f];
        oi += dims->nbu[n] + dims->nbx[n] + dims->ns[n];
    }
    doff[dims->N + 1] = od;
    ioff[dims->N + 1] = oi;
}

extern "C" size_t oqp_qp_bytes(const oqp_dims* dims)
{
    if (!dims) return 0;
    int64_t doff[2], ioff[2];
    (void)doff; (void)ioff;
    const int N = dims->N;
    int64_t od = 0, oi = 0;
    size_t sz[F_COUNT];
    for (int n = 0; n <= N; ++n) {
        stage_sizes(dims, n, sz);
        for (int f = 0; f < F_COUNT; ++f) od += (int64_t)sz[f];
        oi += dims->nbu[n] + dims->nbx[n] + dims->ns[n];
    }
    return align_up(sizeof(oqp_qp), 16) + 2 * align_up((size_t)(N + 2) * sizeof(int64_t), 16) +
           align_up((size_t)od * sizeof(double), 16) + align_up((size_t)oi * sizeof(int), 16);
}

extern "C" int oqp_qp_init(const oqp_dims* dims, void* mem, size_t bytes, oqp_qp** out)
{
    if (!dims || !mem || !out) return fail(OQP_EINVAL, "oqp_qp_init: NULL argument");
    const size_t need = oqp_qp_bytes(dims);
    if (bytes < need) return fail(OQP_ENOMEM, "oqp_qp_init: %zu bytes < %zu", bytes, need);
    if ((uintptr_t)mem % 16) return fail(OQP_EINVAL, "oqp_qp_init: memory not 16-byte aligned");
    if (int rc = check_soft_dims(dims, "oqp_qp_init")) return rc;
    std::memset(mem, 0, need);
    const int N = dims->N;
    char* p = (char*)mem;
    oqp_qp* q = (oqp_qp*)p;
    p += align_up(sizeof(oqp_qp), 16);
    q->dims = dims;
    q->doff = (int64_t*)p;
    p += align_up((size_t)(N + 2) * sizeof(int64_t), 16);
    q->ioff = (int64_t*)p;
    p += align_up((size_t)(N + 2) * sizeof(int64_t), 16);
    qp_offsets(dims, q->doff, q->ioff);
    q->d = (double*)p;
    p += align_up((size_t)q->doff[N + 1] * sizeof(double), 16);
    q->idx = (int*)p;
    *out = q;
    return OQP_OK;
}

double* qp_field(const oqp_qp* q, int n, int f)
{
    size_t sz[F_COUNT];
    stage_sizes(q->dims, n, sz);
    int64_t o = q->doff[n];
    for (int k = 0; k < f; ++k) o += (int64_t)sz[k];
    return q->d + o;
}

static void copy_mat(double* dst, const double* src, int rows, int cols, int ld)
{
    for (int j = 0; j < cols; ++j)
        for (int i = 0; i < rows; ++i) dst[i + (size_t)j * rows] = src[i + (size_t)j * ld];
}

static void copy_sym_lower(double* dst, const double* src, int n, int ld)
{
    for (int j = 0; j < n; ++j)
        for (int i = j; i < n; ++i) {
            double v = src[i + (size_t)j * ld];
            dst[i + (size_t)j * n] = v;
            dst[j + (size_t)i * n] = v;
        }
}

extern "C" int oqp_qp_set_dyn(oqp_qp* q, int n, const double* A, int lda, const double* B, int ldb, const double* b)
{
    if (!q || n < 0 || n >= q->dims->N) return fail(OQP_EINVAL, "oqp_qp_set_dyn: stage %d out of range", n);
    const int nx = q->dims->nx[n], nu = q->dims->nu[n], nxn = q->dims->nx[n + 1];
    if (A && nx > 0) {
        if (lda < nxn || lda < 1) return fail(OQP_EINVAL, "oqp_qp_set_dyn: lda=%d < %d", lda, nxn);
        copy_mat(qp_field(q, n, F_A), A, nxn, nx, lda);
    }
    if (B && nu > 0) {
        if (ldb < nxn || ldb < 1) return fail(OQP_EINVAL, "oqp_qp_set_dyn: ldb=%d < %d", ldb, nxn);
        copy_mat(qp_field(q, n, F_B), B, nxn, nu, ldb);
    }
    if (b) std::memcpy(qp_field(q, n, F_b), b, sizeof(double) * nxn);
    return OQP_OK;
}

extern "C" int oqp_qp_set_cost(oqp_qp* q, int n, const double* Q, int ldq, const double* S, int lds, const double* R,
                               int ldr, const double* qv, const double* rv)
{
    if (!q || n < 0 || n > q->dims->N) return fail(OQP_EINVAL, "oqp_qp_set_cost: stage %d out of range", n);
    const int nx = q->dims->nx[n], nu = q->dims->nu[n];
    if (Q && nx > 0) {
        if (ldq < nx) return fail(OQP_EINVAL, "oqp_qp_set_cost: ldq=%d < %d", ldq, nx);
        copy_sym_lower(qp_field(q, n, F_Q), Q, nx, ldq);
    }
    if (S && nu > 0 && nx > 0) {
        if (lds < nu) return fail(OQP_EINVAL, "oqp_qp_set_cost: lds=%d < %d", lds, nu);
        copy_mat(qp_field(q, n, F_S), S, nu, nx, lds);
    }
    if (R && nu > 0) {
        if (ldr < nu) return fail(OQP_EINVAL, "oqp_qp_set_cost: ldr=%d < %d", ldr, nu);
        copy_sym_lower(qp_field(q, n, F_R), R, nu, ldr);
    }
    if (qv) std::memcpy(qp_field(q, n, F_q), qv, sizeof(double) * nx);
    if (rv) std::memcpy(qp_field(q, n, F_r), rv, sizeof(double) * nu);
    return OQP_OK;
}

static int set_box(oqp_qp* q, int n, const int* idx, const double* lo, const double* hi, bool on_u)
{
    const char* name = on_u ? "oqp_qp_set_box_u" : "oqp_qp_set_box_x";
    if (!q || n < 0 || n > q->dims->N) return fail(OQP_EINVAL, "%s: stage %d out of range", name, n);
    const int nb = on_u ? q->dims->nbu[n] : q->dims->nbx[n];
    const int dim = on_u ? q->dims->nu[n] : q->dims->nx[n];
    if (nb == 0) return OQP_OK;
    if (!idx || !lo || !hi) return fail(OQP_EINVAL, "%s: NULL array", name);
    for (int k = 0; k < nb; ++k) {
        if (idx[k] < 0 || idx[k] >= dim) return fail(OQP_EINVAL, "%s: index %d out of range at stage %d", name, idx[k], n);
        if (!(lo[k] <= hi[k])) return fail(OQP_EINVAL, "%s: lo > hi (or NaN) for bound %d at stage %d", name, k, n);
        for (int k2 = 0; k2 < k; ++k2)
            if (idx[k2] == idx[k]) return fail(OQP_EINVAL, "%s: index %d repeated at stage %d", name, idx[k], n);
    }
    int* dst = q->idx + q->ioff[n] + (on_u ? 0 : q->dims->nbu[n]);
    std::memcpy(dst, idx, sizeof(int) * nb);
    std::memcpy(qp_field(q, n, on_u ? F_lbu : F_lbx), lo, sizeof(double) * nb);
    std::memcpy(qp_field(q, n, on_u ? F_ubu : F_ubx), hi, sizeof(double) * nb);
    return OQP_OK;
}

extern "C" int oqp_qp_set_box_u(oqp_qp* q, int n, const int* idx, const double* lo, const double* hi)
{
    return set_box(q, n, idx, lo, hi, true);
}

extern "C" int oqp_qp_set_box_x(oqp_qp* q, int n, const int* idx, const double* lo, const double* hi)
{
    return set_box(q, n, idx, lo, hi, false);
}

extern "C" int oqp_qp_set_general(oqp_qp* q, int n, const double* D, int ldd, const double* C, int ldc,
                                  const double* lo, const double* hi)
{
    if (!q || n < 0 || n > q->dims->N) return fail(OQP_EINVAL, "oqp_qp_set_general: stage %d out of range", n);
    const int ng = q->dims->ng[n], nu = q->dims->nu[n], nx = q->dims->nx[n];
    if (ng == 0) return OQP_OK;
    if (!lo || !hi) return fail(OQP_EINVAL, "oqp_qp_set_general: NULL bounds");
    for (int k = 0; k < ng; ++k)
        if (!(lo[k] <= hi[k])) return fail(OQP_EINVAL, "oqp_qp_set_general: lo > hi for row %d at stage %d", k, n);
    if (D && nu > 0) {
        if (ldd < ng) return fail(OQP_EINVAL, "oqp_qp_set_general: ldd=%d < %d", ldd, ng);
        copy_mat(qp_field(q, n, F_D), D, ng, nu, ldd);
    }
    if (C && nx > 0) {
        if (ldc < ng) return fail(OQP_EINVAL, "oqp_qp_set_general: ldc=%d < %d", ldc, ng);
        copy_mat(qp_field(q, n, F_C), C, ng, nx, ldc);
    }
    std::memcpy(qp_field(q, n, F_lg), lo, sizeof(double) * ng);
    std::memcpy(qp_field(q, n, F_ug), hi, sizeof(double) * ng);
    return OQP_OK;
}

// Getters mirror the setters: column-major copies into caller arrays with
// the given leading dimensions (Q and R in full); NULL skips a field.
static void copy_out(double* dst, int ld, const double* src, int rows, int cols)
{
    for (int j = 0; j < cols; ++j)
        for (int i = 0; i < rows; ++i) dst[i + (size_t)j * ld] = src[i + (size_t)j * rows];
}

static int check_ld(const char* name, int ld, int rows)
{
    return ld < rows || ld < 1 ? fail(OQP_EINVAL, "%s: leading dimension %d < %d", name, ld, rows) : OQP_OK;
}

extern "C" int oqp_qp_get_dyn(const oqp_qp* q, int n, double* A, int lda, double* B, int ldb, double* b)
{
    if (!q || n < 0 || n >= q->dims->N) return fail(OQP_EINVAL, "oqp_qp_get_dyn: stage %d out of range", n);
    const int nx = q->dims->nx[n], nu = q->dims->nu[n], nxn = q->dims->nx[n + 1];
    if (A && nx > 0) {
        if (check_ld("oqp_qp_get_dyn", lda, nxn)) return OQP_EINVAL;
        copy_out(A, lda, qp_field(q, n, F_A), nxn, nx);
    }
    if (B && nu > 0) {
        if (check_ld("oqp_qp_get_dyn", ldb, nxn)) return OQP_EINVAL;
        copy_out(B, ldb, qp_field(q, n, F_B), nxn, nu);
    }
    if (b) std::memcpy(b, qp_field(q, n, F_b), sizeof(double) * nxn);
    return OQP_OK;
}

extern "C" int oqp_qp_get_cost(const oqp_qp* q, int n, double* Q, int ldq, double* S, int lds, double* R, int ldr,
                               double* qv, double* rv)
{
    if (!q || n < 0 || n > q->dims->N) return fail(OQP_EINVAL, "oqp_qp_get_cost: stage %d out of range", n);
    const int nx = q->dims->nx[n], nu = q->dims->nu[n];
    if (Q && nx > 0) {
        if (check_ld("oqp_qp_get_cost", ldq, nx)) return OQP_EINVAL;
        copy_out(Q, ldq, qp_field(q, n, F_Q), nx, nx);
    }
    if (S && nu > 0 && nx > 0) {
        if (check_ld("oqp_qp_get_cost", lds, nu)) return OQP_EINVAL;
        copy_out(S, lds, qp_field(q, n, F_S), nu, nx);
    }
    if (R && nu > 0) {
        if (check_ld("oqp_qp_get_cost", ldr, nu)) return OQP_EINVAL;
        copy_out(R, ldr, qp_field(q, n, F_R), nu, nu);
    }
    if (qv) std::memcpy(qv, qp_field(q, n, F_q), sizeof(double) * nx);
    if (rv) std::memcpy(rv, qp_field(q, n, F_r), sizeof(double) * nu);
    return OQP_OK;
}

static int get_box(const oqp_qp* q, int n, int* idx, double* lo, double* hi, bool on_u)
{
    if (!q || n < 0 || n > q->dims->N)
        return fail(OQP_EINVAL, "%s: stage %d out of range", on_u ? "oqp_qp_get_box_u" : "oqp_qp_get_box_x", n);
    const int nb = on_u ? q->dims->nbu[n] : q->dims->nbx[n];
    const int* src = q->idx + q->ioff[n] + (on_u ? 0 : q->dims->nbu[n]);
    if (idx) std::memcpy(idx, src, sizeof(int) * nb);
    if (lo) std::memcpy(lo, qp_field(q, n, on_u ? F_lbu : F_lbx), sizeof(double) * nb);
    if (hi) std::memcpy(hi, qp_field(q, n, on_u ? F_ubu : F_ubx), sizeof(double) * nb);
    return OQP_OK;
}

extern "C" int oqp_qp_get_box_u(const oqp_qp* q, int n, int* idx, double* lo, double* hi)
{
    return get_box(q, n, idx, lo, hi, true);
}

extern "C" int oqp_qp_get_box_x(const oqp_qp* q, int n, int* idx, double* lo, double* hi)
{
    return get_box(q, n, idx, lo, hi, false);
}

extern "C" int oqp_qp_get_general(const oqp_qp* q, int n, double* D, int ldd, double* C, int ldc, double* lo,
                                  double* hi)
{
    if (!q || n < 0 || n > q->dims->N) return fail(OQP_EINVAL, "oqp_qp_get_general: stage %d out of range", n);
    const int ng = q->dims->ng[n], nu = q->dims->nu[n], nx = q->dims->nx[n];
    if (ng == 0) return OQP_OK;
    if (D && nu > 0) {
        if (check_ld("oqp_qp_get_general", ldd, ng)) return OQP_EINVAL;
        copy_out(D, ldd, qp_field(q, n, F_D), ng, nu);
    }
    if (C && nx > 0) {
        if (check_ld("oqp_qp_get_general", ldc, ng)) return OQP_EINVAL;
        copy_out(C, ldc, qp_field(q, n, F_C), ng, nx);
    }
    if (lo) std::memcpy(lo, qp_field(q, n, F_lg), sizeof(double) * ng);
    if (hi) std::memcpy(hi, qp_field(q, n, F_ug), sizeof(double) * ng);
    return OQP_OK;
}

// Soft constraints of stage n (Section 2.2): ns_n distinct row indices into
// the stage's rows [box u, box x, general] and the data of each slack pair.
extern "C" int oqp_qp_set_soft(oqp_qp* q, int n, const int* idxs, const double* Zl, const double* Zu,
                               const double* zl, const double* zu, const double* lls, const double* lus)
{
    if (!q || n < 0 || n > q->dims->N) return fail(OQP_EINVAL, "oqp_qp_set_soft: stage %d out of range", n);
    const oqp_dims* d = q->dims;
    const int ns = d->ns[n], nc = d->nbu[n] + d->nbx[n] + d->ng[n];
    if (ns == 0) return OQP_OK;
    if (!idxs || !Zl || !Zu || !zl || !zu || !lls || !lus) return fail(OQP_EINVAL, "oqp_qp_set_soft: NULL argument");
    for (int j = 0; j < ns; ++j) {
        if (idxs[j] < 0 || idxs[j] >= nc)
            return fail(OQP_EINVAL, "oqp_qp_set_soft: row %d out of range [0, %d) at stage %d", idxs[j], nc, n);
        for (int j2 = 0; j2 < j; ++j2)
            if (idxs[j2] == idxs[j]) return fail(OQP_EINVAL, "oqp_qp_set_soft: row %d repeated at stage %d", idxs[j], n);
        if (!(Zl[j] >= 0.0) || !(Zu[j] >= 0.0) || !std::isfinite(Zl[j]) || !std::isfinite(Zu[j]))
            return fail(OQP_EINVAL, "oqp_qp_set_soft: slack Hessian %d at stage %d not finite and >= 0", j, n);
        if (!std::isfinite(zl[j]) || !std::isfinite(zu[j]) || !std::isfinite(lls[j]) || !std::isfinite(lus[j]))
            return fail(OQP_EINVAL, "oqp_qp_set_soft: slack data %d at stage %d not finite", j, n);
    }
    std::memcpy(q->idx + q->ioff[n] + d->nbu[n] + d->nbx[n], idxs, sizeof(int) * ns);
    const double* src[6] = {Zl, Zu, zl, zu, lls, lus};
    for (int f = 0; f < 6; ++f) std::memcpy(qp_field(q, n, F_Zl + f), src[f], sizeof(double) * ns);
    return OQP_OK;
}

extern "C" int oqp_qp_get_soft(const oqp_qp* q, int n, int* idxs, double* Zl, double* Zu, double* zl, double* zu,
                               double* lls, double* lus)
{
    if (!q || n < 0 || n > q->dims->N) return fail(OQP_EINVAL, "oqp_qp_get_soft: stage %d out of range", n);
    const oqp_dims* d = q->dims;
    const int ns = d->ns[n];
    if (idxs) std::memcpy(idxs, q->idx + q->ioff[n] + d->nbu[n] + d->nbx[n], sizeof(int) * ns);
    double* dst[6] = {Zl, Zu, zl, zu, lls, lus};
    for (int f = 0; f < 6; ++f)
        if (dst[f]) std::memcpy(dst[f], qp_field(q, n, F_Zl + f), sizeof(double) * ns);
    return OQP_OK;
}

// ---------------------------------------------------------------------------
// arguments
// ---------------------------------------------------------------------------

extern "C" void oqp_arg_default(oqp_arg* a, int mode)
{
    if (!a) return;
    std::memset(a, 0, sizeof(*a));
    a->mode = (mode == OQP_MODE_MIXED || mode == OQP_MODE_ABS || mode == OQP_MODE_ROBUST || mode == OQP_MODE_BALANCE)
                  ? mode
                  : OQP_MODE_F64;
    const double tol = a->mode == OQP_MODE_MIXED ? 1e-6 : 1e-8;
    a->tol_stat = a->tol_eq = a->tol_ineq = a->tol_comp = tol;
    a->iter_max = 100;
    a->alpha_min = 1e-10;
    a->gamma = 0.995;
    a->lam_min = 1e-16;
    a->t_min = 1e-16;
    a->reg_prim = 0.0;
    a->corr_ratio = 10.0;
    // refinement steps: a few in balance mode, more in robust mode (Section
    // 4.2), as many on the mixed path
    a->ir_max = (a->mode == OQP_MODE_MIXED || a->mode == OQP_MODE_ROBUST) ? 4 : (a->mode == OQP_MODE_BALANCE ? 2 : 0);
    a->ir_tol = 1e-10;
    a->warm_start = 0;
    a->cond_N = 0;
}

int check_arg(const oqp_arg* a)
{
    if (!a) return fail(OQP_EINVAL, "NULL oqp_arg");
    if (a->mode != OQP_MODE_F64 && a->mode != OQP_MODE_MIXED && a->mode != OQP_MODE_ABS && a->mode != OQP_MODE_ROBUST &&
        a->mode != OQP_MODE_BALANCE)
        return fail(OQP_EINVAL, "unknown mode %d", a->mode);
    if (a->iter_max < 0 || !(a->gamma > 0.0 && a->gamma <= 1.0) || a->warm_start < 0 || a->warm_start > 2 ||
        a->ir_max < 0 || a->cond_N < 0 || (a->warm_start != 0 && a->cond_N != 0))
        return fail(OQP_EINVAL, "bad oqp_arg field (iter_max, gamma, warm_start or cond_N)");
    return OQP_OK;
}

// ---------------------------------------------------------------------------
// batch
// ---------------------------------------------------------------------------

// An instance as solved (the QP itself, or its condensed QP) and as given
// (the original horizon and record sizes; equal to the solved ones without
// condensing).
struct Inst {
    int variant;    // kernel group (see select_kernel)
    int nx, nu, ng; // padded stage sizes of the device records
    int N;          // horizon of the solved QP
    int nuN;        // inputs of its terminal stage (unpadded)
    int nc;
    int dims_off;   // into dims pool: 5 * (oN+1) ints (nx, nu, nbu, nbx, ng) of the original QP
    int slot_off;   // into slot pool: per-stage user constraint -> padded slot (original records)
    int64_t data;   // doubles
    int64_t iter;   // doubles
    int64_t work;   // doubles
    int oN;              // horizon of the original QP
    int onx, onu, ong;   // record sizes of the original QP
    int64_t odata;       // original data records (into hdata/ddata, or the condensing regions)
    int64_t oiter;       // original-layout iterate records
    int soft;            // soft layout (the batch has slacks)
    int nsoft;           // slack pairs of the instance
    int soft_off;        // into soft pool: ns per stage (oN+1), then the device slot of each slack
};

struct oqp_batch {
    int count;
    int nvar;
    oqp_arg arg;
    void* stream;
    int loaded;
    int solved;
    int has_step;
    int iter_dirty;  // host iterate records changed since the last upload
    // extra caller streams for concurrent kernel groups, with fork/join events
    int naux;
    void* aux[OQP_BATCH_MAX_AUX];
    void* ev_fork;
    void* ev_join[OQP_BATCH_MAX_AUX];
    int iter_valid;  // the device iterate records hold an iterate (a solve ran, or one was set)
    // host side
    Inst* inst;
    int* dims_pool;
    int* slot_pool;
    int soft;        // some instance has slacks: every instance solved by the soft kernel builds
    int* soft_pool;
    InstDesc* hdesc;
    DevStat* hstat;
    double* hdata;
    double* hiter;
    double* hstep;
    int* vstart;
    int* vcount;
    // device side
    InstDesc* ddesc;
    DevStat* dstat;
    double* ddata;
    double* diter;
    double* dwork;
    double* dstep;
    // sizes (doubles)
    int64_t n_data, n_iter, n_work;
    // partial condensing (cond != 0): original QPs, expanded iterates, the
    // stage tables and work items of the condensing kernels
    int cond;
    int cond_fetched;
    int n_items;
    size_t cond_lds;
    int64_t n_odata, n_oiter;
    double* hodata;
    double* hoiter;
    oqp::CondDesc* hcdesc;
    oqp::CondItem* hitems;
    int* htab;
    double* dodata;
    double* doiter;
    oqp::CondDesc* dcdesc;
    oqp::CondItem* ditems;
    int* dtab;
};

static int pick_variant_max(int mx, int mu, int mg)
{
    int best = -1;
    long best_cost = 0;
    for (int v = 0; v < oqp::variant_count(); ++v) {
        int nx, nu, ng;
        oqp::variant_dims(v, &nx, &nu, &ng);
        if (nx < mx || nu < mu || ng < mg) continue;
        long nz = nx + nu;
        long cost = nz * nz * (nx + nz) + (long)ng * nz * nz;
        if (best < 0 || cost < best_cost) {
            best = v;
            best_cost = cost;
        }
    }
    return best;
}

int pick_variant(const oqp_dims* d)
{
    int mx = 0, mu = 0, mg = 0;
    for (int n = 0; n <= d->N; ++n) {
        if (d->nx[n] > mx) mx = d->nx[n];
        if (d->nu[n] > mu) mu = d->nu[n];
        if (d->ng[n] > mg) mg = d->ng[n];
    }
    return pick_variant_max(mx, mu, mg);
}

// Kernel groups: 0..variant_count()-1 are the one-wave variants; the block
// kernel builds follow (stage-block bound 32, 64 or 256, without or with
// general rows), then the wide-stage kernel (batches only: stages beyond the
// block kernel's limits).  One-wave variants are used up to a stage block of
// g_wave_max_nz, larger instances go to the block kernel, padded only to
// their own maximum stage sizes.
// 24 by default: the 32-wide variants win on batches of their own size, but
// in uneven mixes their two extra kernel groups split the launches (uneven
// 4096 on one stream 482 -> 532 ms, mixed 781 -> 832 ms, serving saturation
// 7.6k -> 7.0k/s), so they are used when the bound is raised
// (oqp_set_wave_max, or the autotuner on same-size batches)
static int g_wave_max_nz = 24;
// one-wave variants allowed (bit v: variant v); the others' instances go to
// the block kernel (set by the schedule autotuner per kernel group)
static unsigned g_variant_mask = ~0u;
// batches launch the block-group instances needing more than half a CU's LDS
// apart from the rest (off: one launch per group)
static int g_lds_split = 1;
static const int kBlockZ[6] = {32, 32, 64, 64, 256, 256};
static const int kBlockG[6] = {0, 64, 0, 64, 0, 64};
static constexpr size_t kMaxLds = 160 * 1024;

// the wide-stage kernel's group follows the block kernel builds
int group_count() { return oqp::variant_count() + 7; }
static int wide_group() { return oqp::variant_count() + 6; }

static void dims_max(const oqp_dims* d, int* mx, int* mu, int* mg)
{
    *mx = *mu = *mg = 0;
    for (int n = 0; n <= d->N; ++n) {
        if (d->nx[n] > *mx) *mx = d->nx[n];
        if (d->nu[n] > *mu) *mu = d->nu[n];
        if (d->ng[n] > *mg) *mg = d->ng[n];
    }
}

static int select_block_max(int mx, int mu, int mg, KSel* out);

// kernel for an instance whose largest stage sizes are mx, mu, mg
static int select_kernel_max(int mx, int mu, int mg, KSel* out)
{
    const int v = pick_variant_max(mx, mu, mg);
    if (v >= 0) {
        int nx, nu, ng;
        oqp::variant_dims(v, &nx, &nu, &ng);
        if (nx + nu <= g_wave_max_nz && ((g_variant_mask >> v) & 1u)) {
            *out = KSel{v, nx, nu, ng};
            return OQP_OK;
        }
    }
    return select_block_max(mx, mu, mg, out);
}

// the block kernel build for the largest stage sizes
static int select_block_max(int mx, int mu, int mg, KSel* out)
{
    if (mx < 1) mx = 1;
    const int zm = oqp::block_zmax(mx + mu);
    // one thread per row and per constraint slot; the u block is solved on
    // one wave
    if (zm == 0 || mg > 64 || mu > 64 || mx + mu + mg > 256) return -1;
    if ((size_t)oqp::block_lds_bytes(mx, mu, mg) > kMaxLds) return -1;
    const int b = (zm == 256 ? 4 : (zm == 64 ? 2 : 0)) + (mg > 0 ? 1 : 0);
    *out = KSel{oqp::variant_count() + b, mx, mu, mg};
    return OQP_OK;
}

int select_kernel(const oqp_dims* d, KSel* out)
{
    int mx, mu, mg;
    dims_max(d, &mx, &mu, &mg);
    return select_kernel_max(mx, mu, mg, out);
}

// ---------------------------------------------------------------------------
// partial condensing: blocks and condensed stage sizes (Section 3.5)
// ---------------------------------------------------------------------------

static int cond_horizon(int N, int cond_N) { return cond_N < N ? cond_N : N; }

// first stage of block b of N2 (block N2 starts at N): near-equal blocks, the
// first N mod N2 of them one stage longer
static int cond_start(int N, int N2, int b)
{
    const int q = N / N2, r = N % N2;
    return b * q + (b < r ? b : r);
}

struct CStage {
    int nx, nu, nbu, nbx, ng;
};

// sizes of condensed stage b (b = N2: the terminal stage N)
static CStage cond_stage(const oqp_dims* d, int N2, int b)
{
    const int s0 = b < N2 ? cond_start(d->N, N2, b) : d->N;
    const int s1 = b < N2 ? cond_start(d->N, N2, b + 1) : d->N + 1;
    CStage c{d->nx[s0], 0, 0, d->nbx[s0], 0};
    for (int n = s0; n < s1; ++n) {
        c.nu += d->nu[n];
        c.nbu += d->nbu[n];
        c.ng += d->ng[n] + (n > s0 ? d->nbx[n] : 0);
    }
    return c;
}

extern "C" size_t oqp_pcond_dims_bytes(const oqp_dims* d, int cond_N)
{
    if (!d || cond_N < 1) return 0;
    return oqp_dims_bytes(cond_horizon(d->N, cond_N));
}

extern "C" int oqp_pcond_dims(const oqp_dims* d, int cond_N, void* mem, size_t bytes, oqp_dims** out)
{
    if (!d || !out || cond_N < 1) return fail(OQP_EINVAL, "oqp_pcond_dims: bad argument (cond_N=%d)", cond_N);
    const int N2 = cond_horizon(d->N, cond_N);
    oqp_dims* c;
    int rc = oqp_dims_init(mem, bytes, N2, &c);
    if (rc) return rc;
    for (int b = 0; b <= N2; ++b) {
        const CStage s = cond_stage(d, N2, b);
        c->nx[b] = s.nx;
        c->nu[b] = s.nu;
        c->nbu[b] = s.nbu;
        c->nbx[b] = s.nbx;
        c->ng[b] = s.ng;
    }
    *out = c;
    return OQP_OK;
}

// The QP solved for an instance: the QP itself or, with cond_N > 0, its
// condensed QP; plus the record sizes of the original QP.
struct SolveShape {
    int N;
    KSel ks;
    int onx, onu, ong;
};

static constexpr size_t kMaxCondLds = 160 * 1024;

// Kernel for the largest stage sizes (every mode has the same kernels: the
// array-algorithm builds exist for the one-wave variants and the block
// kernel alike).  Stages beyond the block kernel's limits go to the
// wide-stage kernel: FP64 delta formulation without refinement, no slacks.
static int select_for_mode(int mx, int mu, int mg, const oqp_arg* a, int soft, KSel* out)
{
    if (select_kernel_max(mx, mu, mg, out) == OQP_OK) return OQP_OK;
    if (a->mode != OQP_MODE_F64 || a->ir_max != 0 || soft) return -1;
    if (mx < 1) mx = 1;
    if ((size_t)oqp::wide_lds_bytes(mx, mu, mg) > kMaxLds) return -1;
    *out = KSel{wide_group(), mx, mu, mg};
    return OQP_OK;
}

static int solve_shape(const oqp_dims* d, const oqp_arg* arg, int soft, SolveShape* sh, int i)
{
    const int cond_N = arg->cond_N;
    if (cond_N <= 0) {
        sh->N = d->N;
        int mx, mu, mg;
        dims_max(d, &mx, &mu, &mg);
        if (select_for_mode(mx, mu, mg, arg, soft, &sh->ks))
            return fail(OQP_EINVAL,
                        "batch: no kernel covers the stage sizes of instance %d (stages beyond the block kernel's "
                        "limits need the FP64 mode without refinement)",
                        i);
        sh->onx = sh->ks.nx;
        sh->onu = sh->ks.nu;
        sh->ong = sh->ks.ng;
        return OQP_OK;
    }
    dims_max(d, &sh->onx, &sh->onu, &sh->ong);
    const int N2 = cond_horizon(d->N, cond_N);
    int cx = 0, cu = 0, cg = 0;
    for (int b = 0; b <= N2; ++b) {
        const CStage c = cond_stage(d, N2, b);
        if (c.nx > cx) cx = c.nx;
        if (c.nu > cu) cu = c.nu;
        if (c.ng > cg) cg = c.ng;
    }
    sh->N = N2;
    if (select_for_mode(cx, cu, cg, arg, 0, &sh->ks))
        return fail(OQP_EINVAL,
                    "batch: no kernel covers the condensed stage sizes of instance %d (nx %d, nu %d, ng %d; stages "
                    "beyond the block kernel's limits need the FP64 mode without refinement)",
                    i, cx, cu, cg);
    if ((size_t)oqp::cond_lds_bytes(sh->onx, sh->onu, sh->ks.nx + sh->ks.nu) > kMaxCondLds)
        return fail(OQP_EINVAL, "batch: condensed stage of instance %d too large for the condensing kernel", i);
    return OQP_OK;
}

extern "C" int oqp_set_wave_max(int nz)
{
    if (nz < 0 || nz > 64) return fail(OQP_EINVAL, "oqp_set_wave_max: stage block bound must be in [0, 64]");
    g_wave_max_nz = nz;
    return OQP_OK;
}

extern "C" int oqp_get_wave_max(void) { return g_wave_max_nz; }

extern "C" int oqp_set_variant_mask(unsigned mask)
{
    g_variant_mask = mask;
    return OQP_OK;
}

extern "C" unsigned oqp_get_variant_mask(void) { return g_variant_mask; }

extern "C" int oqp_set_lds_split(int on)
{
    if (on != 0 && on != 1) return fail(OQP_EINVAL, "oqp_set_lds_split: 0 or 1");
    g_lds_split = on;
    return OQP_OK;
}

extern "C" int oqp_get_lds_split(void) { return g_lds_split; }

// A block-kernel instance whose LDS block exceeds half of a CU's LDS keeps
// the CU to itself; the others can share it two by two.
static constexpr size_t kLdsHalf = kMaxLds / 2;

static bool lds_big(const InstDesc& d)
{
    return (size_t)oqp::block_lds_bytes(d.nx, d.nu, d.ng) > kLdsHalf;
}

// Launch the instances [desc, desc + count) of kernel group g.  A block
// group's launch takes the LDS size of its largest instance; with split_lds
// (a batch, which orders them first) a leading run of instances needing more
// than half a CU's LDS is launched on its own and the rest in a second launch
// on the same stream, sized so that two of its workgroups share a CU.  The
// server keeps one launch: its requests come in arrival order, and a launch
// of a few large ones would hold up the rest of the stream.
int group_launch(int g, int km, const InstDesc* desc, const InstDesc* hdesc, int count, const double* data,
                 double* iter, double* work, double* step, DevStat* stat, const oqp::KParams& P, void* stream,
                 bool split_lds)
{
    const int nv = oqp::variant_count();
    if (g < nv) return oqp::variant_launch(g, km, desc, count, data, iter, work, step, stat, P, stream);
    if (g == wide_group()) {
        if (km != oqp::KM_F64) return -1;  // FP64 only (the plan refuses other modes)
        size_t lds = 0;
        for (int i = 0; i < count; ++i) {
            const size_t b = (size_t)oqp::wide_lds_bytes(hdesc[i].nx, hdesc[i].nu, hdesc[i].ng);
            if (b > lds) lds = b;
        }
        return oqp::wide_launch(desc, count, data, iter, work, step, stat, P, lds, stream);
    }
    int split = 0;
    while (split_lds && g_lds_split && split < count && lds_big(hdesc[split])) ++split;
    if (split == count) split = 0;
    const int parts[3] = {0, split, count};
    for (int p = split > 0 ? 0 : 1; p < 2; ++p) {
        const int lo = parts[p], hi = parts[p + 1];
        size_t lds = 0;
        for (int i = lo; i < hi; ++i) {
            const size_t b = (size_t)oqp::block_lds_bytes(hdesc[i].nx, hdesc[i].nu, hdesc[i].ng);
            if (b > lds) lds = b;
        }
        const int rc = oqp::block_launch(kBlockZ[g - nv], kBlockG[g - nv], km, desc + lo, hi - lo, data, iter, work,
                                         step, stat, P, lds, stream);
        if (rc) return rc;
    }
    return 0;
}

// relative cost of an instance, for ordering a launch largest first
double inst_cost(int N, int nx, int nu)
{
    const double nz = nx + nu;
    return (N + 1.0) * nz * nz * (nx + nz);
}

struct Plan {
    size_t host_bytes, dev_bytes;
    // host offsets
    size_t h_inst, h_dims, h_slot, h_desc, h_stat, h_data, h_iter, h_step, h_vstart, h_vcount;
    size_t h_odata, h_oiter, h_cdesc, h_items, h_tab;
    // device offsets
    size_t d_desc, d_stat, d_data, d_iter, d_work, d_step;
    size_t d_odata, d_oiter, d_cdesc, d_items, d_tab;
    int64_t n_data, n_iter, n_work, n_odata, n_oiter;
    int n_dims, n_slot, n_items, n_tab;
    size_t cond_lds;
    int soft;
    size_t h_soft;
    int n_soft;
};

// A batch with slacks anywhere (every instance then takes the soft builds):
// FP64 delta formulation, without condensing.
static int batch_soft(const oqp_dims* const* dims, int count, const oqp_arg* arg, int* soft)
{
    *soft = 0;
    for (int i = 0; i < count; ++i)
        if (dims[i] && dims_soft(dims[i])) *soft = 1;
    if (!*soft) return OQP_OK;
    if (arg->mode != OQP_MODE_F64 || arg->cond_N != 0 || arg->ir_max != 0)
        return fail(OQP_EINVAL, "batch: soft constraints need the FP64 mode without refinement and no condensing");
    for (int i = 0; i < count; ++i)
        if (dims[i] && check_soft_dims(dims[i], "batch")) return OQP_EINVAL;
    return OQP_OK;
}

static int make_plan(const oqp_dims* const* dims, int count, const oqp_arg* arg, Plan* pl)
{
    const int cond_N = arg->cond_N;
    if (!dims || count < 1) return fail(OQP_EINVAL, "batch: count must be >= 1");
    const int nv = group_count();
    const int cond = cond_N > 0;
    int64_t nd = 0, ni = 0, nw = 0, nod = 0, noi = 0;
    int ndims = 0, nslot = 0, nitems = 0, ntab = 0, nsoft = 0;
    size_t clds = 0;
    int soft = 0;
    if (int rc = batch_soft(dims, count, arg, &soft)) return rc;
    for (int i = 0; i < count; ++i) {
        const oqp_dims* d = dims[i];
        if (!d) return fail(OQP_EINVAL, "batch: dims[%d] is NULL", i);
        SolveShape sh;
        int rc = solve_shape(d, arg, soft, &sh, i);
        if (rc) return rc;
        const Layout L = oqp::make_layout(sh.ks.nx, sh.ks.nu, sh.ks.ng, soft);
        if (soft) {
            nsoft += d->N + 1;
            for (int n = 0; n <= d->N; ++n) nsoft += d->ns[n];
        }
        nd += (int64_t)(sh.N + 1) * L.SREC;
        ni += (int64_t)(sh.N + 1) * L.IREC;
        nw += (int64_t)(sh.N + 1) * L.WREC;
        ndims += 5 * (d->N + 1);
        for (int n = 0; n <= d->N; ++n) nslot += d->nbu[n] + d->nbx[n] + d->ng[n];
        if (cond) {
            const Layout Lo = oqp::make_layout(sh.onx, sh.onu, sh.ong);
            nod += (int64_t)(d->N + 1) * Lo.SREC;
            noi += (int64_t)(d->N + 1) * Lo.IREC;
            nitems += sh.N + 1;
            ntab += 4 * (d->N + 1) + sh.N + 1;
            const size_t lb = (size_t)oqp::cond_lds_bytes(sh.onx, sh.onu, sh.ks.nx + sh.ks.nu);
            if (lb > clds) clds = lb;
        }
    }
    size_t h = 0;
    h = align_up(h + sizeof(oqp_batch), 64);
    pl->h_inst = h; h = align_up(h + sizeof(Inst) * count, 64);
    pl->h_dims = h; h = align_up(h + sizeof(int) * ndims, 64);
    pl->h_slot = h; h = align_up(h + sizeof(int) * (nslot + 1), 64);
    pl->h_vstart = h; h = align_up(h + sizeof(int) * nv, 64);
    pl->h_vcount = h; h = align_up(h + sizeof(int) * nv, 64);
    pl->h_desc = h; h = align_up(h + sizeof(InstDesc) * count, 64);
    pl->h_stat = h; h = align_up(h + sizeof(DevStat) * count, 64);
    pl->h_data = h; h = align_up(h + sizeof(double) * nd, 64);
    pl->h_iter = h; h = align_up(h + sizeof(double) * ni, 64);
    pl->h_step = h; h = align_up(h + sizeof(double) * ni, 64);
    pl->h_odata = h; h = align_up(h + sizeof(double) * nod, 64);
    pl->h_oiter = h; h = align_up(h + sizeof(double) * noi, 64);
    pl->h_cdesc = h; h = align_up(h + sizeof(oqp::CondDesc) * (cond ? count : 0), 64);
    pl->h_items = h; h = align_up(h + sizeof(oqp::CondItem) * nitems, 64);
    pl->h_tab = h; h = align_up(h + sizeof(int) * ntab, 64);
    pl->h_soft = h; h = align_up(h + sizeof(int) * nsoft, 64);
    pl->host_bytes = h;
    size_t g = 0;
    pl->d_desc = g; g = align_up(g + sizeof(InstDesc) * count, 256);
    pl->d_stat = g; g = align_up(g + sizeof(DevStat) * count, 256);
    pl->d_data = g; g = align_up(g + sizeof(double) * nd, 256);
    pl->d_iter = g; g = align_up(g + sizeof(double) * ni, 256);
    pl->d_work = g; g = align_up(g + sizeof(double) * nw, 256);
    pl->d_step = g; g = align_up(g + sizeof(double) * ni, 256);
    pl->d_odata = g; g = align_up(g + sizeof(double) * nod, 256);
    pl->d_oiter = g; g = align_up(g + sizeof(double) * noi, 256);
    pl->d_cdesc = g; g = align_up(g + sizeof(oqp::CondDesc) * (cond ? count : 0), 256);
    pl->d_items = g; g = align_up(g + sizeof(oqp::CondItem) * nitems, 256);
    pl->d_tab = g; g = align_up(g + sizeof(int) * ntab, 256);
    pl->dev_bytes = g;
    pl->n_data = nd; pl->n_iter = ni; pl->n_work = nw;
    pl->n_odata = nod; pl->n_oiter = noi;
    pl->n_dims = ndims; pl->n_slot = nslot;
    pl->n_items = nitems; pl->n_tab = ntab;
    pl->cond_lds = clds;
    pl->soft = soft;
    pl->n_soft = nsoft;
    return OQP_OK;
}

extern "C" int oqp_batch_bytes(const oqp_dims* const* dims, int count, const oqp_arg* arg, size_t* host_bytes,
                               size_t* dev_bytes)
{
    int rc = check_arg(arg);
    if (rc) return rc;
    Plan pl;
    rc = make_plan(dims, count, arg, &pl);
    if (rc) return rc;
    if (host_bytes) *host_bytes = pl.host_bytes;
    if (dev_bytes) *dev_bytes = pl.dev_bytes;
    return OQP_OK;
}

static const Layout inst_layout(const Inst& in) { return oqp::make_layout(in.nx, in.nu, in.ng, in.soft); }
// records of the QP as given (the solved records without condensing)
static const Layout orig_layout(const Inst& in) { return oqp::make_layout(in.onx, in.onu, in.ong, in.soft); }

extern "C" int oqp_batch_init(const oqp_dims* const* dims, int count, const oqp_arg* arg, void* host_mem,
                              size_t host_bytes, void* dev_mem, size_t dev_bytes, void* stream, oqp_batch** out)
{
    int rc = check_arg(arg);
    if (rc) return rc;
    if (!host_mem || !dev_mem || !out) return fail(OQP_EINVAL, "oqp_batch_init: NULL argument");
    if ((uintptr_t)host_mem % 16) return fail(OQP_EINVAL, "oqp_batch_init: host memory not 16-byte aligned");
    if ((uintptr_t)dev_mem % 256) return fail(OQP_EINVAL, "oqp_batch_init: device memory not 256-byte aligned");
    Plan pl;
    rc = make_plan(dims, count, arg, &pl);
    if (rc) return rc;
    if (host_bytes < pl.host_bytes) return fail(OQP_ENOMEM, "oqp_batch_init: host %zu < %zu", host_bytes, pl.host_bytes);
    if (dev_bytes < pl.dev_bytes) return fail(OQP_ENOMEM, "oqp_batch_init: device %zu < %zu", dev_bytes, pl.dev_bytes);
    char* h = (char*)host_mem;
    char* g = (char*)dev_mem;
    oqp_batch* b = (oqp_batch*)h;
    std::memset(b, 0, sizeof(*b));
    b->count = count;
    b->nvar = group_count();
    b->arg = *arg;
    b->stream = stream;
    b->inst = (Inst*)(h + pl.h_inst);
    b->dims_pool = (int*)(h + pl.h_dims);
    b->slot_pool = (int*)(h + pl.h_slot);
    b->vstart = (int*)(h + pl.h_vstart);
    b->vcount = (int*)(h + pl.h_vcount);
    b->hdesc = (InstDesc*)(h + pl.h_desc);
    b->hstat = (DevStat*)(h + pl.h_stat);
    b->hdata = (double*)(h + pl.h_data);
    b->hiter = (double*)(h + pl.h_iter);
    b->hstep = (double*)(h + pl.h_step);
    b->ddesc = (InstDesc*)(g + pl.d_desc);
    b->dstat = (DevStat*)(g + pl.d_stat);
    b->ddata = (double*)(g + pl.d_data);
    b->diter = (double*)(g + pl.d_iter);
    b->dwork = (double*)(g + pl.d_work);
    b->dstep = (double*)(g + pl.d_step);
    b->n_data = pl.n_data;
    b->n_iter = pl.n_iter;
    b->n_work = pl.n_work;
    b->cond = arg->cond_N > 0;
    b->n_items = pl.n_items;
    b->cond_lds = pl.cond_lds;
    b->n_odata = pl.n_odata;
    b->n_oiter = pl.n_oiter;
    b->hodata = (double*)(h + pl.h_odata);
    b->hoiter = (double*)(h + pl.h_oiter);
    b->hcdesc = (oqp::CondDesc*)(h + pl.h_cdesc);
    b->hitems = (oqp::CondItem*)(h + pl.h_items);
    b->htab = (int*)(h + pl.h_tab);
    b->dodata = (double*)(g + pl.d_odata);
    b->doiter = (double*)(g + pl.d_oiter);
    b->dcdesc = (oqp::CondDesc*)(g + pl.d_cdesc);
    b->ditems = (oqp::CondItem*)(g + pl.d_items);
    b->dtab = (int*)(g + pl.d_tab);
    b->soft = pl.soft;
    b->soft_pool = (int*)(h + pl.h_soft);
    // instances, grouped by variant
    int doff = 0, soff = 0, ssoff = 0;
    for (int v = 0; v < b->nvar; ++v) b->vcount[v] = 0;
    for (int i = 0; i < count; ++i) {
        Inst& in = b->inst[i];
        const oqp_dims* d = dims[i];
        SolveShape sh;
        solve_shape(d, arg, pl.soft, &sh, i);
        const KSel& ks = sh.ks;
        in.variant = ks.group;
        in.nx = ks.nx;
        in.nu = ks.nu;
        in.ng = ks.ng;
        in.N = sh.N;
        in.nuN = d->nu[d->N];  // the condensed terminal stage keeps the original one's inputs
        in.oN = d->N;
        in.onx = sh.onx;
        in.onu = sh.onu;
        in.ong = sh.ong;
        in.dims_off = doff;
        in.slot_off = soff;
        int nc = 0;
        for (int n = 0; n <= d->N; ++n) {
            b->dims_pool[doff + 0 * (d->N + 1) + n] = d->nx[n];
            b->dims_pool[doff + 1 * (d->N + 1) + n] = d->nu[n];
            b->dims_pool[doff + 2 * (d->N + 1) + n] = d->nbu[n];
            b->dims_pool[doff + 3 * (d->N + 1) + n] = d->nbx[n];
            b->dims_pool[doff + 4 * (d->N + 1) + n] = d->ng[n];
            nc += d->nbu[n] + d->nbx[n] + d->ng[n];
        }
        in.nc = nc;
        doff += 5 * (d->N + 1);
        soff += nc;
        in.soft = pl.soft;
        in.nsoft = 0;
        in.soft_off = ssoff;
        if (pl.soft) {
            for (int n = 0; n <= d->N; ++n) {
                b->soft_pool[ssoff + n] = d->ns[n];
                in.nsoft += d->ns[n];
            }
            ssoff += d->N + 1 + in.nsoft;
        }
        b->vcount[in.variant]++;
    }
    int acc = 0;
    for (int v = 0; v < b->nvar; ++v) {
        b->vstart[v] = acc;
        acc += b->vcount[v];
    }
    // region offsets in group order; within a group, largest instances first
    int64_t od = 0, oi = 0, ow = 0;
    int* order = (int*)b->hstat;  // count ints of scratch: the status block is only filled by a fetch
    for (int v = 0; v < b->nvar; ++v) {
        int k = 0;
        for (int i = 0; i < count; ++i)
            if (b->inst[i].variant == v) order[k++] = i;
        // block groups: instances needing more than half a CU's LDS first
        // (group_launch gives them a launch of their own)
        const bool blk = v >= oqp::variant_count();
        std::stable_sort(order, order + k, [&](int x, int y) {
            const Inst& a = b->inst[x];
            const Inst& c = b->inst[y];
            if (blk) {
                const bool ba = (size_t)oqp::block_lds_bytes(a.nx, a.nu, a.ng) > kLdsHalf;
                const bool bc = (size_t)oqp::block_lds_bytes(c.nx, c.nu, c.ng) > kLdsHalf;
                if (ba != bc) return ba;
            }
            return inst_cost(a.N, a.nx, a.nu) > inst_cost(c.N, c.nx, c.nu);
        });
        for (int q = 0; q < k; ++q) {
            const int i = order[q];
            Inst& in = b->inst[i];
            const Layout L = inst_layout(in);
            in.data = od;
            in.iter = oi;
            in.work = ow;
            od += (int64_t)(in.N + 1) * L.SREC;
            oi += (int64_t)(in.N + 1) * L.IREC;
            ow += (int64_t)(in.N + 1) * L.WREC;
            InstDesc& ds = b->hdesc[b->vstart[v] + q];
            ds.data = in.data;
            ds.iter = in.iter;
            ds.work = in.work;
            ds.N = in.N;
            ds.nc = in.nc + in.nsoft;  // one-sided rows / 2: constraint rows and slack bounds
            ds.index = i;
            ds.resume = 0;
            ds.nx = in.nx;
            ds.nu = in.nu;
            ds.ng = in.ng;
            ds.itcap = 0;
            ds.nuN = in.nuN;
            ds.pad = 0;
        }
    }
    // original records: the solved ones, or (condensing) regions of their own
    int64_t ood = 0, ooi = 0;
    int ot = 0, oit = 0;
    for (int i = 0; i < count; ++i) {
        Inst& in = b->inst[i];
        if (!b->cond) {
            in.odata = in.data;
            in.oiter = in.iter;
            continue;
        }
        const Layout Lo = orig_layout(in);
        in.odata = ood;
        in.oiter = ooi;
        ood += (int64_t)(in.oN + 1) * Lo.SREC;
        ooi += (int64_t)(in.oN + 1) * Lo.IREC;
        oqp::CondDesc& cd = b->hcdesc[i];
        std::memset(&cd, 0, sizeof(cd));
        cd.odata = in.odata;
        cd.oiter = in.oiter;
        cd.cdata = in.data;
        cd.citer = in.iter;
        cd.N = in.oN;
        cd.N2 = in.N;
        cd.tab = ot;
        cd.onx = in.onx;
        cd.onu = in.onu;
        cd.ong = in.ong;
        cd.cnx = in.nx;
        cd.cnu = in.nu;
        cd.cng = in.ng;
        const oqp_dims* d = dims[i];
        for (int n = 0; n <= in.oN; ++n) {
            b->htab[ot++] = d->nx[n];
            b->htab[ot++] = d->nu[n];
            b->htab[ot++] = d->nbx[n];
            b->htab[ot++] = d->ng[n];
        }
        for (int c = 0; c <= in.N; ++c) b->htab[ot++] = c < in.N ? cond_start(in.oN, in.N, c) : in.oN;
        for (int c = 0; c <= in.N; ++c) b->hitems[oit++] = oqp::CondItem{i, c};
    }
    hipStream_t hs = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(b->ddesc, b->hdesc, sizeof(InstDesc) * count, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess && b->cond)
        e = hipMemcpyAsync(b->dcdesc, b->hcdesc, sizeof(oqp::CondDesc) * count, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess && b->cond)
        e = hipMemcpyAsync(b->ditems, b->hitems, sizeof(oqp::CondItem) * oit, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess && b->cond) e = hipMemcpyAsync(b->dtab, b->htab, sizeof(int) * ot, hipMemcpyHostToDevice, hs);
    if (e != hipSuccess) return fail(OQP_EDEVICE, "oqp_batch_init: hipMemcpyAsync: %s", hipGetErrorString(e));
    *out = b;
    return OQP_OK;
}

extern "C" int oqp_batch_init_static(const oqp_dims* const* dims, int count, const oqp_arg* arg, void* host_mem,
                                     size_t host_bytes, void* stream, oqp_batch** out)
{
    int rc = check_arg(arg);
    if (rc) return rc;
    if (!host_mem || !out) return fail(OQP_EINVAL, "oqp_batch_init_static: NULL argument");
    Plan pl;
    rc = make_plan(dims, count, arg, &pl);
    if (rc) return rc;
    void* region = nullptr;
    size_t cap = 0;
    rc = static_dev_region(&region, &cap);
    if (rc) return rc;
    if (pl.dev_bytes > cap)
        return fail(OQP_ENOMEM, "oqp_batch_init_static: the batch needs %zu device bytes, the static region holds %zu",
                    pl.dev_bytes, cap);
    return oqp_batch_init(dims, count, arg, host_mem, host_bytes, region, cap, stream, out);
}

static inline const int* inst_dims(const oqp_batch* b, const Inst& in, int which)
{
    return b->dims_pool + in.dims_off + which * (in.oN + 1);
}

// Pack a QP into N+1 padded stage records (L.SREC doubles each) at dst and
// fill the map from user constraint order to padded slot (nc entries).
int pack_records(const oqp_qp* q, const Layout& L, double* dst, int* slots, int* sslots)
{
    const oqp_dims* qd = q->dims;
    const int N = qd->N;
    const int NX = L.NX, NU = L.NU, NZ = L.NZ;
    int so = 0, sso = 0;
    for (int n = 0; n <= N; ++n) {
        const int so0 = so;
        double* r = dst + (int64_t)n * L.SREC;
        std::memset(r, 0, sizeof(double) * L.SREC);
        const int nx = qd->nx[n], nu = qd->nu[n], nxn = n < N ? qd->nx[n + 1] : 0, ng = qd->ng[n];
        if (nx > NX || nu > NU || ng > L.NG || nxn > NX) return fail(OQP_EINVAL, "pack: stage %d exceeds the variant", n);
        // F = [B A]
        if (n < N) {
            const double* A = qp_field(q, n, F_A);
            const double* B = qp_field(q, n, F_B);
            const double* bb = qp_field(q, n, F_b);
            for (int j = 0; j < nu; ++j)
                for (int i2 = 0; i2 < nxn; ++i2) r[L.D_F + i2 + j * NX] = B[i2 + (size_t)j * nxn];
            for (int j = 0; j < nx; ++j)
                for (int i2 = 0; i2 < nxn; ++i2) r[L.D_F + i2 + (NU + j) * NX] = A[i2 + (size_t)j * nxn];
            for (int i2 = 0; i2 < nxn; ++i2) r[L.D_b + i2] = bb[i2];
        }
        // H = [[R, S], [S', Q]] padded with unit diagonal
        {
            const double* Q = qp_field(q, n, F_Q);
            const double* S = qp_field(q, n, F_S);
            const double* R = qp_field(q, n, F_R);
            double* H = r + L.D_H;
            for (int j = 0; j < nu; ++j)
                for (int i2 = 0; i2 < nu; ++i2) H[i2 + j * NZ] = R[i2 + (size_t)j * nu];
            for (int j = 0; j < nx; ++j)
                for (int i2 = 0; i2 < nu; ++i2) {
                    const double sv = S[i2 + (size_t)j * nu];
                    H[i2 + (NU + j) * NZ] = sv;
                    H[(NU + j) + i2 * NZ] = sv;
                }
            for (int j = 0; j < nx; ++j)
                for (int i2 = 0; i2 < nx; ++i2) H[(NU + i2) + (NU + j) * NZ] = Q[i2 + (size_t)j * nx];
            for (int j = nu; j < NU; ++j) H[j + j * NZ] = 1.0;
            for (int j = NU + nx; j < NZ; ++j) H[j + j * NZ] = 1.0;
            const double* qv = qp_field(q, n, F_q);
            const double* rv = qp_field(q, n, F_r);
            for (int j = 0; j < nu; ++j) r[L.D_g + j] = rv[j];
            for (int j = 0; j < nx; ++j) r[L.D_g + NU + j] = qv[j];
        }
        // boxes
        {
            const int nbu = qd->nbu[n], nbx = qd->nbx[n];
            const int* iu = q->idx + q->ioff[n];
            const int* ix = iu + nbu;
            const double* lbu = qp_field(q, n, F_lbu);
            const double* ubu = qp_field(q, n, F_ubu);
            const double* lbx = qp_field(q, n, F_lbx);
            const double* ubx = qp_field(q, n, F_ubx);
            for (int k = 0; k < nbu; ++k) {
                const int c = iu[k];
                r[L.D_bm + c] = 1.0;
                r[L.D_blo + c] = lbu[k];
                r[L.D_bhi + c] = ubu[k];
                slots[so++] = c;
            }
            for (int k = 0; k < nbx; ++k) {
                const int c = NU + ix[k];
                r[L.D_bm + c] = 1.0;
                r[L.D_blo + c] = lbx[k];
                r[L.D_bhi + c] = ubx[k];
                slots[so++] = c;
            }
        }
        // general rows
        if (ng > 0) {
            const double* D = qp_field(q, n, F_D);
            const double* C = qp_field(q, n, F_C);
            const double* lg = qp_field(q, n, F_lg);
            const double* ug = qp_field(q, n, F_ug);
            for (int k = 0; k < ng; ++k) {
                for (int j = 0; j < nu; ++j) r[L.D_G + k + j * L.NG] = D[k + (size_t)j * ng];
                for (int j = 0; j < nx; ++j) r[L.D_G + k + (NU + j) * L.NG] = C[k + (size_t)j * ng];
                r[L.D_gm + k] = 1.0;
                r[L.D_glo + k] = lg[k];
                r[L.D_ghi + k] = ug[k];
                slots[so++] = NZ + k;
            }
        }
        // soft constraints: slot mask and the slack data of each softened slot
        const int ns = qd->ns[n];
        if (ns > 0) {
            if (!L.SOFT) return fail(OQP_EINVAL, "pack: stage %d has slacks but the records have no slack blocks", n);
            const int* is = q->idx + q->ioff[n] + qd->nbu[n] + qd->nbx[n];
            const int offs[6] = {L.D_Zl, L.D_Zu, L.D_zl, L.D_zu, L.D_lls, L.D_lus};
            for (int j = 0; j < ns; ++j) {
                const int c = slots[so0 + is[j]];
                r[L.D_sm + c] = 1.0;
                for (int f = 0; f < 6; ++f) r[offs[f] + c] = qp_field(q, n, F_Zl + f)[j];
                if (sslots) sslots[sso++] = c;
            }
        }
    }
    return OQP_OK;
}

static int pack_instance(oqp_batch* b, int i, const oqp_qp* q)
{
    const Inst& in = b->inst[i];
    const Layout L = orig_layout(in);
    const int* nxv = inst_dims(b, in, 0);
    const int* nuv = inst_dims(b, in, 1);
    const int* nbuv = inst_dims(b, in, 2);
    const int* nbxv = inst_dims(b, in, 3);
    const int* ngv = inst_dims(b, in, 4);
    const oqp_dims* qd = q->dims;
    if (qd->N != in.oN) return fail(OQP_EINVAL, "oqp_batch_load: qp %d horizon differs from its dims", i);
    for (int n = 0; n <= in.oN; ++n)
        if (qd->nx[n] != nxv[n] || qd->nu[n] != nuv[n] || qd->nbu[n] != nbuv[n] || qd->nbx[n] != nbxv[n] ||
            qd->ng[n] != ngv[n])
            return fail(OQP_EINVAL, "oqp_batch_load: qp %d sizes differ from its dims at stage %d", i, n);
    int* sp = in.soft ? b->soft_pool + in.soft_off : nullptr;
    for (int n = 0; n <= in.oN; ++n)
        if (qd->ns[n] != (sp ? sp[n] : 0))
            return fail(OQP_EINVAL, "oqp_batch_load: qp %d slack count differs from its dims at stage %d", i, n);
    return pack_records(q, L, (b->cond ? b->hodata : b->hdata) + in.odata, b->slot_pool + in.slot_off,
                        sp ? sp + in.oN + 1 : nullptr);
}

extern "C" int oqp_batch_load(oqp_batch* b, const oqp_qp* const* qps)
{
    if (!b || !qps) return fail(OQP_EINVAL, "oqp_batch_load: NULL argument");
    for (int i = 0; i < b->count; ++i) {
        if (!qps[i]) return fail(OQP_EINVAL, "oqp_batch_load: qp %d is NULL", i);
        int rc = pack_instance(b, i, qps[i]);
        if (rc) return rc;
    }
    hipError_t e = b->cond ? hipMemcpyAsync(b->dodata, b->hodata, sizeof(double) * b->n_odata,
                                            hipMemcpyHostToDevice, (hipStream_t)b->stream)
                           : hipMemcpyAsync(b->ddata, b->hdata, sizeof(double) * b->n_data, hipMemcpyHostToDevice,
                                            (hipStream_t)b->stream);
    if (e != hipSuccess) return fail(OQP_EDEVICE, "oqp_batch_load: hipMemcpyAsync: %s", hipGetErrorString(e));
    b->loaded = 1;
    b->solved = 0;
    b->cond_fetched = 0;
    return OQP_OK;
}

oqp::KParams make_params(const oqp_arg& a, int mode, double tau)
{
    oqp::KParams P{};
    P.tol_stat = a.tol_stat;
    P.tol_eq = a.tol_eq;
    P.tol_ineq = a.tol_ineq;
    P.tol_comp = a.tol_comp;
    P.alpha_min = a.alpha_min;
    P.gamma = a.gamma;
    P.lam_min = a.lam_min;
    P.t_min = a.t_min;
    P.reg_prim = a.reg_prim;
    P.corr_ratio = a.corr_ratio;
    P.ir_tol = a.ir_tol;
    P.tau = tau;
    P.iter_max = a.iter_max;
    P.ir_max = a.ir_max;
    P.mode = mode;
    P.warm = mode == oqp::KMODE_SOLVE ? a.warm_start : 0;
    return P;
}

int kernel_build(int mode)
{
    if (mode == OQP_MODE_MIXED) return oqp::KM_MIXED;
    if (mode == OQP_MODE_ABS) return oqp::KM_ABS;
    if (mode == OQP_MODE_ROBUST) return oqp::KM_ROBUST;
    if (mode == OQP_MODE_BALANCE) return oqp::KM_BALANCE;
    return oqp::KM_F64;
}

// Stream of kernel group v: the first non-empty group (in launch order) on
// the batch stream, the others round-robin over the extra streams.
static void* group_stream(const oqp_batch* b, int v)
{
    if (b->naux == 0) return b->stream;
    int k = 0;
    for (int u = b->nvar - 1; u > v; --u)
        if (b->vcount[u] > 0) ++k;
    return k == 0 ? b->stream : b->aux[(k - 1) % b->naux];
}

static int launch_all(oqp_batch* b, const oqp::KParams& P)
{
    const int km = b->soft ? oqp::KM_SOFT : kernel_build(b->arg.mode);
    hipError_t e = hipSuccess;
    if (b->naux > 0) {
        e = hipEventRecord((hipEvent_t)b->ev_fork, (hipStream_t)b->stream);
        for (int k = 0; k < b->naux && e == hipSuccess; ++k)
            e = hipStreamWaitEvent((hipStream_t)b->aux[k], (hipEvent_t)b->ev_fork, 0);
        if (e != hipSuccess) return fail(OQP_EDEVICE, "batch fork: %s", hipGetErrorString(e));
    }
    // block-kernel groups first: they hold the largest instances
    for (int pass = 0; pass < 2; ++pass) {
        oqp::KParams Pp = P;
        if (pass == 1) {
            if (!(km == oqp::KM_MIXED && P.mode == oqp::KMODE_SOLVE)) break;
            // FP64 kernels pick up the instances the mixed kernels handed over
            // (from their iterate when it is finite, else from a cold start)
            Pp.mode = oqp::KMODE_FALLBACK;
            Pp.ir_max = 0;  // the fallback is the plain FP64 path (no refinement)
            Pp.warm = 0;
        }
        for (int k = 0; k < b->nvar; ++k) {
            const int v = b->nvar - 1 - k;
            if (b->vcount[v] == 0) continue;
            int rc = group_launch(v, pass == 0 ? km : oqp::KM_F64, b->ddesc + b->vstart[v], b->hdesc + b->vstart[v],
                                  b->vcount[v], b->ddata, b->diter, b->dwork, b->dstep, b->dstat, Pp,
                                  group_stream(b, v), true);
            if (rc) return fail(OQP_EDEVICE, "kernel launch failed for group %d", v);
        }
    }
    // join: later work on the batch stream waits for every extra stream
    for (int k = 0; k < b->naux && e == hipSuccess; ++k) {
        e = hipEventRecord((hipEvent_t)b->ev_join[k], (hipStream_t)b->aux[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent((hipStream_t)b->stream, (hipEvent_t)b->ev_join[k], 0);
    }
    if (e != hipSuccess) return fail(OQP_EDEVICE, "batch join: %s", hipGetErrorString(e));
    return OQP_OK;
}

extern "C" int oqp_batch_set_streams(oqp_batch* b, void* const* streams, int n)
{
    if (!b || n < 0 || n > OQP_BATCH_MAX_AUX || (n > 0 && !streams))
        return fail(OQP_EINVAL, "oqp_batch_set_streams: bad argument (n=%d, at most %d)", n, OQP_BATCH_MAX_AUX);
    int rc = oqp_batch_release(b);
    if (rc) return rc;
    if (n == 0) return OQP_OK;
    hipError_t e = hipEventCreateWithFlags((hipEvent_t*)&b->ev_fork, hipEventDisableTiming);
    for (int k = 0; k < n && e == hipSuccess; ++k) {
        b->ev_join[k] = nullptr;
        e = hipEventCreateWithFlags((hipEvent_t*)&b->ev_join[k], hipEventDisableTiming);
        b->aux[k] = streams[k];
        b->naux = k + 1;
    }
    if (e != hipSuccess) {
        oqp_batch_release(b);
        return fail(OQP_EDEVICE, "oqp_batch_set_streams: %s", hipGetErrorString(e));
    }
    return OQP_OK;
}

extern "C" int oqp_batch_release(oqp_batch* b)
{
    if (!b) return fail(OQP_EINVAL, "oqp_batch_release: NULL batch");
    if (b->naux > 0 || b->ev_fork) {
        hipError_t e = hipStreamSynchronize((hipStream_t)b->stream);
        if (e != hipSuccess) return fail(OQP_EDEVICE, "oqp_batch_release: %s", hipGetErrorString(e));
    }
    for (int k = 0; k < b->naux; ++k)
        if (b->ev_join[k]) (void)hipEventDestroy((hipEvent_t)b->ev_join[k]);
    if (b->ev_fork) (void)hipEventDestroy((hipEvent_t)b->ev_fork);
    b->ev_fork = nullptr;
    b->naux = 0;
    return OQP_OK;
}

extern "C" int oqp_batch_solve(oqp_batch* b)
{
    if (!b) return fail(OQP_EINVAL, "oqp_batch_solve: NULL batch");
    if (!b->loaded) return fail(OQP_ESTATE, "oqp_batch_solve: no data loaded");
    // warm start from iterates set on the host
    if (b->arg.warm_start != 0 && !b->iter_valid && !b->iter_dirty)
        return fail(OQP_ESTATE, "oqp_batch_solve: warm start without an iterate (solve once or set one)");
    if (b->arg.warm_start != 0 && b->iter_dirty) {
        hipError_t e = hipMemcpyAsync(b->diter, b->hiter, sizeof(double) * b->n_iter, hipMemcpyHostToDevice,
                                      (hipStream_t)b->stream);
        if (e != hipSuccess) return fail(OQP_EDEVICE, "oqp_batch_solve: %s", hipGetErrorString(e));
        b->iter_dirty = 0;
    }
    // partial condensing: original records -> condensed records, every solve
    if (b->cond && oqp::cond_launch(0, b->dcdesc, b->ditems, b->n_items, b->dtab, b->dodata, b->ddata, nullptr,
                                    nullptr, b->cond_lds, b->stream))
        return fail(OQP_EDEVICE, "oqp_batch_solve: condensing kernel launch failed");
    int rc = launch_all(b, make_params(b->arg, oqp::KMODE_SOLVE, 0.0));
    if (rc) return rc;
    if (b->cond && oqp::cond_launch(1, b->dcdesc, b->ditems, b->n_items, b->dtab, b->dodata, nullptr, b->diter,
                                    b->doiter, 0, b->stream))
        return fail(OQP_EDEVICE, "oqp_batch_solve: expansion kernel launch failed");
    b->solved = 1;
    b->iter_valid = 1;
    return OQP_OK;
}

extern "C" int oqp_batch_set_arg(oqp_batch* b, const oqp_arg* a)
{
    if (!b) return fail(OQP_EINVAL, "oqp_batch_set_arg: NULL batch");
    int rc = check_arg(a);
    if (rc) return rc;
    if (a->mode != b->arg.mode) return fail(OQP_EINVAL, "oqp_batch_set_arg: mode cannot change");
    if (a->cond_N != b->arg.cond_N) return fail(OQP_EINVAL, "oqp_batch_set_arg: cond_N cannot change");
    b->arg = *a;
    return OQP_OK;
}

extern "C" int oqp_batch_fetch(oqp_batch* b)
{
    if (!b) return fail(OQP_EINVAL, "oqp_batch_fetch: NULL batch");
    hipStream_t s = (hipStream_t)b->stream;
    hipError_t e = hipMemcpyAsync(b->hstat, b->dstat, sizeof(DevStat) * b->count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = b->cond ? hipMemcpyAsync(b->hoiter, b->doiter, sizeof(double) * b->n_oiter, hipMemcpyDeviceToHost, s)
                    : hipMemcpyAsync(b->hiter, b->diter, sizeof(double) * b->n_iter, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && b->has_step)
        e = hipMemcpyAsync(b->hstep, b->dstep, sizeof(double) * b->n_iter, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return fail(OQP_EDEVICE, "oqp_batch_fetch: %s", hipGetErrorString(e));
    return OQP_OK;
}

extern "C" int oqp_batch_sync(oqp_batch* b)
{
    if (!b) return fail(OQP_EINVAL, "oqp_batch_sync: NULL batch");
    hipError_t e = hipStreamSynchronize((hipStream_t)b->stream);
    if (e != hipSuccess) return fail(OQP_EDEVICE, "oqp_batch_sync: %s", hipGetErrorString(e));
    return OQP_OK;
}

extern "C" int oqp_batch_get_stat(const oqp_batch* b, int i, oqp_stat* st)
{
    if (!b || !st || i < 0 || i >= b->count) return fail(OQP_EINVAL, "oqp_batch_get_stat: bad argument");
    const DevStat& d = b->hstat[i];
    st->status = d.status;
    st->iters = d.iters;
    st->ir_steps = d.ir_steps;
    st->fell_back_f64 = d.fell_back;
    st->qr_refactors = d.qr_refactors;
    st->mu = d.mu;
    for (int k = 0; k < 4; ++k) st->res[k] = d.res[k];
    return OQP_OK;
}

// Copy between padded iterate records (N+1 of L.IREC doubles at rec) and the
// user layout; dims5 holds nx, nu, nbu, nbx, ng, each N+1 entries.
void iterate_user_copy(const int* dims5, int N, const int* slots, const Layout& L, double* rec, bool to_user,
                       double* u, double* x, double* pi, double* ll, double* lu, double* tl, double* tu)
{
    const int* nxv = dims5;
    const int* nuv = dims5 + (N + 1);
    const int* nbuv = dims5 + 2 * (N + 1);
    const int* nbxv = dims5 + 3 * (N + 1);
    const int* ngv = dims5 + 4 * (N + 1);
    int ou = 0, ox = 0, op = 0, oc = 0;
    for (int n = 0; n <= N; ++n) {
        double* r = rec + (int64_t)n * L.IREC;
        const int nu = nuv[n], nx = nxv[n];
        for (int j = 0; j < nu; ++j) {
            if (u) { if (to_user) u[ou + j] = r[L.I_z + j]; else r[L.I_z + j] = u[ou + j]; }
        }
        for (int j = 0; j < nx; ++j) {
            if (x) { if (to_user) x[ox + j] = r[L.I_z + L.NU + j]; else r[L.I_z + L.NU + j] = x[ox + j]; }
        }
        if (n > 0) {
            for (int j = 0; j < nx; ++j) {
                if (pi) { if (to_user) pi[op + j] = r[L.I_pi + j]; else r[L.I_pi + j] = pi[op + j]; }
            }
            op += nx;
        }
        const int nc = nbuv[n] + nbxv[n] + ngv[n];
        for (int k = 0; k < nc; ++k) {
            const int c = slots[oc + k];
            double* vals[4] = {ll, lu, tl, tu};
            const int offs[4] = {L.I_ll, L.I_lu, L.I_tl, L.I_tu};
            for (int a2 = 0; a2 < 4; ++a2) {
                if (!vals[a2]) continue;
                if (to_user) vals[a2][oc + k] = r[offs[a2] + c];
                else r[offs[a2] + c] = vals[a2][oc + k];
            }
        }
        ou += nu;
        ox += nx;
        oc += nc;
    }
}

// region: original-layout iterate records (hiter/hstep, or hoiter with condensing)
static void user_copy(const oqp_batch* b, int i, double* region, bool to_user, double* u, double* x, double* pi,
                      double* ll, double* lu, double* tl, double* tu)
{
    const Inst& in = b->inst[i];
    iterate_user_copy(b->dims_pool + in.dims_off, in.oN, b->slot_pool + in.slot_off, orig_layout(in),
                      region + in.oiter, to_user, u, x, pi, ll, lu, tl, tu);
}

bool dims5_match(const int* d5, int N, const oqp_dims* d)
{
    if (!d || d->N != N) return false;
    for (int n = 0; n <= N; ++n)
        if (d5[n] != d->nx[n] || d5[(N + 1) + n] != d->nu[n] || d5[2 * (N + 1) + n] != d->nbu[n] ||
            d5[3 * (N + 1) + n] != d->nbx[n] || d5[4 * (N + 1) + n] != d->ng[n])
            return false;
    return true;
}

bool batch_dims_match(const oqp_batch* b, int i, const oqp_dims* d)
{
    if (!b || i < 0 || i >= b->count) return false;
    const Inst& in = b->inst[i];
    return dims5_match(b->dims_pool + in.dims_off, in.oN, d);
}

extern "C" int oqp_batch_get_sol(const oqp_batch* b, int i, double* u, double* x, double* pi, double* lam_l,
                                 double* lam_u, double* t_l, double* t_u)
{
    if (!b || i < 0 || i >= b->count) return fail(OQP_EINVAL, "oqp_batch_get_sol: bad argument");
    user_copy(b, i, b->cond ? b->hoiter : b->hiter, true, u, x, pi, lam_l, lam_u, t_l, t_u);
    return OQP_OK;
}

extern "C" int oqp_batch_set_iterate(oqp_batch* b, int i, const double* u, const double* x, const double* pi,
                                     const double* lam_l, const double* lam_u, const double* t_l, const double* t_u)
{
    if (!b || i < 0 || i >= b->count || !u || !x || !pi || !lam_l || !lam_u || !t_l || !t_u)
        return fail(OQP_EINVAL, "oqp_batch_set_iterate: bad argument");
    if (b->cond) return fail(OQP_ESTATE, "oqp_batch_set_iterate: not available with partial condensing");
    const Inst& in = b->inst[i];
    const Layout L = inst_layout(in);
    std::memset(b->hiter + in.iter, 0, sizeof(double) * (size_t)(in.N + 1) * L.IREC);
    user_copy(b, i, b->hiter, false, (double*)u, (double*)x, (double*)pi, (double*)lam_l, (double*)lam_u,
              (double*)t_l, (double*)t_u);
    b->iter_dirty = 1;
    return OQP_OK;
}

// Slack blocks between N+1 iterate records (soft layout L) at rec and the
// user layout (stage by stage in idxs order); soft: ns per stage (N+1
// entries), then the device slot of every slack.
void soft_iterate_copy(const int* soft, int N, const Layout& L, double* rec, bool to_user, double* const vals[6])
{
    const int* cs = soft + N + 1;
    const int offs[6] = {L.I_sl, L.I_su, L.I_lsl, L.I_lsu, L.I_tsl, L.I_tsu};
    int o = 0;
    for (int n = 0; n <= N; ++n) {
        double* r = rec + (int64_t)n * L.IREC;
        for (int j = 0; j < soft[n]; ++j, ++o)
            for (int f = 0; f < 6; ++f) {
                if (!vals[f]) continue;
                if (to_user) vals[f][o] = r[offs[f] + cs[o]];
                else r[offs[f] + cs[o]] = vals[f][o];
            }
    }
}

static void soft_user_copy(const oqp_batch* b, int i, double* region, bool to_user, double* const vals[6])
{
    const Inst& in = b->inst[i];
    soft_iterate_copy(b->soft_pool + in.soft_off, in.oN, orig_layout(in), region + in.oiter, to_user, vals);
}

extern "C" int oqp_batch_get_soft_sol(const oqp_batch* b, int i, double* s_l, double* s_u, double* lam_sl,
                                      double* lam_su, double* t_sl, double* t_su)
{
    if (!b || i < 0 || i >= b->count) return fail(OQP_EINVAL, "oqp_batch_get_soft_sol: bad argument");
    if (!b->soft) return OQP_OK;
    double* const v[6] = {s_l, s_u, lam_sl, lam_su, t_sl, t_su};
    soft_user_copy(b, i, b->hiter, true, v);
    return OQP_OK;
}

extern "C" int oqp_batch_set_soft_iterate(oqp_batch* b, int i, const double* s_l, const double* s_u,
                                          const double* lam_sl, const double* lam_su, const double* t_sl,
                                          const double* t_su)
{
    if (!b || i < 0 || i >= b->count) return fail(OQP_EINVAL, "oqp_batch_set_soft_iterate: bad argument");
    if (!b->soft) return fail(OQP_ESTATE, "oqp_batch_set_soft_iterate: the batch has no slacks");
    if (b->inst[i].nsoft > 0 && (!s_l || !s_u || !lam_sl || !lam_su || !t_sl || !t_su))
        return fail(OQP_EINVAL, "oqp_batch_set_soft_iterate: NULL argument");
    double* const v[6] = {(double*)s_l, (double*)s_u, (double*)lam_sl, (double*)lam_su, (double*)t_sl,
                          (double*)t_su};
    soft_user_copy(b, i, b->hiter, false, v);
    b->iter_dirty = 1;
    return OQP_OK;
}

extern "C" int oqp_batch_get_soft_step(const oqp_batch* b, int i, double* ds_l, double* ds_u, double* dlam_sl,
                                       double* dlam_su, double* dt_sl, double* dt_su)
{
    if (!b || i < 0 || i >= b->count) return fail(OQP_EINVAL, "oqp_batch_get_soft_step: bad argument");
    if (!b->has_step) return fail(OQP_ESTATE, "oqp_batch_get_soft_step: no Newton step computed");
    if (!b->soft) return OQP_OK;
    double* const v[6] = {ds_l, ds_u, dlam_sl, dlam_su, dt_sl, dt_su};
    soft_user_copy(b, i, b->hstep, true, v);
    return OQP_OK;
}

extern "C" int oqp_batch_nsoft(const oqp_batch* b, int i)
{
    if (!b || i < 0 || i >= b->count) return fail(OQP_EINVAL, "oqp_batch_nsoft: bad argument");
    return b->inst[i].nsoft;
}

extern "C" int oqp_batch_newton(oqp_batch* b, double tau)
{
    if (!b) return fail(OQP_EINVAL, "oqp_batch_newton: NULL batch");
    if (!b->loaded) return fail(OQP_ESTATE, "oqp_batch_newton: no data loaded");
    if (b->cond) return fail(OQP_ESTATE, "oqp_batch_newton: not available with partial condensing");
    hipError_t e = hipMemcpyAsync(b->diter, b->hiter, sizeof(double) * b->n_iter, hipMemcpyHostToDevice,
                                  (hipStream_t)b->stream);
    if (e != hipSuccess) return fail(OQP_EDEVICE, "oqp_batch_newton: %s", hipGetErrorString(e));
    b->iter_dirty = 0;
    b->iter_valid = 1;
    int rc = launch_all(b, make_params(b->arg, oqp::KMODE_NEWTON, tau));
    if (rc) return rc;
    b->has_step = 1;
    return OQP_OK;
}

extern "C" int oqp_batch_get_step(const oqp_batch* b, int i, double* du, double* dx, double* dpi, double* dll,
                                  double* dlu, double* dtl, double* dtu)
{
    if (!b || i < 0 || i >= b->count) return fail(OQP_EINVAL, "oqp_batch_get_step: bad argument");
    if (!b->has_step) return fail(OQP_ESTATE, "oqp_batch_get_step: no Newton step computed");
    user_copy(b, i, b->hstep, true, du, dx, dpi, dll, dlu, dtl, dtu);
    return OQP_OK;
}

extern "C" int oqp_batch_fetch_cond(oqp_batch* b)
{
    if (!b) return fail(OQP_EINVAL, "oqp_batch_fetch_cond: NULL batch");
    if (!b->cond) return fail(OQP_ESTATE, "oqp_batch_fetch_cond: the batch does not condense");
    if (!b->solved) return fail(OQP_ESTATE, "oqp_batch_fetch_cond: no solve enqueued");
    hipError_t e = hipMemcpyAsync(b->hdata, b->ddata, sizeof(double) * b->n_data, hipMemcpyDeviceToHost,
                                  (hipStream_t)b->stream);
    if (e != hipSuccess) return fail(OQP_EDEVICE, "oqp_batch_fetch_cond: %s", hipGetErrorString(e));
    b->cond_fetched = 1;
    return OQP_OK;
}

// Unpack the condensed records of instance i (host copy) into a QP with the
// condensed dims: the inverse of pack_records for one record layout.
extern "C" int oqp_batch_get_cond_qp(const oqp_batch* b, int i, oqp_qp* q)
{
    if (!b || !q || i < 0 || i >= b->count) return fail(OQP_EINVAL, "oqp_batch_get_cond_qp: bad argument");
    if (!b->cond || !b->cond_fetched) return fail(OQP_ESTATE, "oqp_batch_get_cond_qp: no condensed QP fetched");
    const Inst& in = b->inst[i];
    const oqp_dims* qd = q->dims;
    const int N2 = in.N, N = in.oN;
    const int* d5 = b->dims_pool + in.dims_off;
    oqp_dims od{N, (int*)d5, (int*)d5 + (N + 1), (int*)d5 + 2 * (N + 1), (int*)d5 + 3 * (N + 1),
                (int*)d5 + 4 * (N + 1)};
    if (qd->N != N2) return fail(OQP_EINVAL, "oqp_batch_get_cond_qp: horizon %d, expected %d", qd->N, N2);
    for (int c = 0; c <= N2; ++c) {
        const CStage cs = cond_stage(&od, N2, c);
        if (qd->nx[c] != cs.nx || qd->nu[c] != cs.nu || qd->nbu[c] != cs.nbu || qd->nbx[c] != cs.nbx ||
            qd->ng[c] != cs.ng)
            return fail(OQP_EINVAL, "oqp_batch_get_cond_qp: stage %d sizes differ from the condensed QP", c);
    }
    const Layout L = inst_layout(in);
    const int NU = L.NU, NZ = L.NZ, NX = L.NX, NG = L.NG;
    for (int n = 0; n <= N2; ++n) {
        const double* r = b->hdata + in.data + (int64_t)n * L.SREC;
        const int nx = qd->nx[n], nu = qd->nu[n], ng = qd->ng[n], nxn = n < N2 ? qd->nx[n + 1] : 0;
        if (n < N2) {
            double* A = qp_field(q, n, F_A);
            double* B = qp_field(q, n, F_B);
            double* bb = qp_field(q, n, F_b);
            for (int j = 0; j < nx; ++j)
                for (int k = 0; k < nxn; ++k) A[k + (size_t)j * nxn] = r[L.D_F + k + (NU + j) * NX];
            for (int j = 0; j < nu; ++j)
                for (int k = 0; k < nxn; ++k) B[k + (size_t)j * nxn] = r[L.D_F + k + j * NX];
            for (int k = 0; k < nxn; ++k) bb[k] = r[L.D_b + k];
        }
        double* Q = qp_field(q, n, F_Q);
        double* S = qp_field(q, n, F_S);
        double* R = qp_field(q, n, F_R);
        const double* H = r + L.D_H;
        for (int j = 0; j < nu; ++j)
            for (int k = 0; k < nu; ++k) R[k + (size_t)j * nu] = H[k + j * NZ];
        for (int j = 0; j < nx; ++j)
            for (int k = 0; k < nu; ++k) S[k + (size_t)j * nu] = H[k + (NU + j) * NZ];
        for (int j = 0; j < nx; ++j)
            for (int k = 0; k < nx; ++k) Q[k + (size_t)j * nx] = H[(NU + k) + (NU + j) * NZ];
        double* rv = qp_field(q, n, F_r);
        double* qv = qp_field(q, n, F_q);
        for (int j = 0; j < nu; ++j) rv[j] = r[L.D_g + j];
        for (int j = 0; j < nx; ++j) qv[j] = r[L.D_g + NU + j];
        // boxes in increasing component order
        int* iu = q->idx + q->ioff[n];
        int* ix = iu + qd->nbu[n];
        double* lbu = qp_field(q, n, F_lbu);
        double* ubu = qp_field(q, n, F_ubu);
        double* lbx = qp_field(q, n, F_lbx);
        double* ubx = qp_field(q, n, F_ubx);
        int k = 0;
        for (int j = 0; j < nu; ++j)
            if (r[L.D_bm + j] != 0.0) {
                if (k == qd->nbu[n]) return fail(OQP_EINVAL, "oqp_batch_get_cond_qp: input boxes exceed nbu");
                iu[k] = j;
                lbu[k] = r[L.D_blo + j];
                ubu[k] = r[L.D_bhi + j];
                ++k;
            }
        k = 0;
        for (int j = 0; j < nx; ++j)
            if (r[L.D_bm + NU + j] != 0.0) {
                if (k == qd->nbx[n]) return fail(OQP_EINVAL, "oqp_batch_get_cond_qp: state boxes exceed nbx");
                ix[k] = j;
                lbx[k] = r[L.D_blo + NU + j];
                ubx[k] = r[L.D_bhi + NU + j];
                ++k;
            }
        if (ng > 0) {
            double* D = qp_field(q, n, F_D);
            double* C = qp_field(q, n, F_C);
            double* lg = qp_field(q, n, F_lg);
            double* ug = qp_field(q, n, F_ug);
            for (int g = 0; g < ng; ++g) {
                for (int j = 0; j < nu; ++j) D[g + (size_t)j * ng] = r[L.D_G + g + j * NG];
                for (int j = 0; j < nx; ++j) C[g + (size_t)j * ng] = r[L.D_G + g + (NU + j) * NG];
                lg[g] = r[L.D_glo + g];
                ug[g] = r[L.D_ghi + g];
            }
        }
    }
    return OQP_OK;
}

extern "C" int oqp_batch_variant(const oqp_batch* b, int i, int* nx, int* nu, int* ng)
{
    if (!b || i < 0 || i >= b->count) return fail(OQP_EINVAL, "oqp_batch_variant: bad argument");
    const Inst& in = b->inst[i];
    if (nx) *nx = in.nx;
    if (nu) *nu = in.nu;
    if (ng) *ng = in.ng;
    return in.variant;
}

extern "C" int oqp_variant_count(void) { return oqp::variant_count(); }

extern "C" int oqp_variant_dims(int v, int* nx, int* nu, int* ng)
{
    if (v < 0 || v >= oqp::variant_count()) return fail(OQP_EINVAL, "oqp_variant_dims: no variant %d", v);
    oqp::variant_dims(v, nx, nu, ng);
    return OQP_OK;
}

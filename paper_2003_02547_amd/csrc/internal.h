// Internal declarations shared by the C-ABI implementation units.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/oqp.h"
#include "layout.h"

struct oqp_dims {
    int N;
    int* nx;
    int* nu;
    int* nbu;
    int* nbx;
    int* ng;
    int* ns;  // soft constraints (slack pairs) per stage
};

// Per-stage double block of a host QP: A, B, b, Q, S, R, q, r, lbu, ubu, lbx, ubx, D, C, lg, ug, and the
// slack data Zl, Zu, zl, zu, lls, lus (ns each).
enum { F_A, F_B, F_b, F_Q, F_S, F_R, F_q, F_r, F_lbu, F_ubu, F_lbx, F_ubx, F_D, F_C, F_lg, F_ug,
       F_Zl, F_Zu, F_zl, F_zu, F_lls, F_lus, F_COUNT };

struct oqp_qp {
    const oqp_dims* dims;
    int64_t* doff;  // (N+2) stage offsets into d
    int64_t* ioff;  // (N+2) stage offsets into idx (idxbu, idxbx, then idxs)
    double* d;
    int* idx;
};

namespace oqp {
int variant_count();
void variant_dims(int v, int* nx, int* nu, int* ng);
int variant_launch(int v, int km, const InstDesc* desc, int count, const double* data, double* iter, double* work,
                   double* step, DevStat* stat, const KParams& P, void* stream);
int block_lds_bytes(int nx, int nu, int ng);
int block_zmax(int nz);
int block_launch(int zm, int gm, int km, const InstDesc* desc, int count, const double* data, double* iter,
                 double* work, double* step, DevStat* stat, const KParams& P, size_t lds_bytes, void* stream);
// wide-stage kernel (stages beyond the block kernel's limits; FP64)
int wide_lds_bytes(int nx, int nu, int ng);
int wide_launch(const InstDesc* desc, int count, const double* data, double* iter, double* work, double* step,
                DevStat* stat, const KParams& P, size_t lds_bytes, void* stream);
// partial condensing (expand = 0: original data -> condensed data records;
// expand = 1: condensed iterate -> original-layout iterate records)
int cond_lds_bytes(int onx, int onu, int cnz);
int cond_launch(int expand, const CondDesc* cds, const CondItem* items, int nitems, const int* tab,
                const double* odata, double* cdata, const double* citer, double* oiter, size_t lds_bytes,
                void* stream);
}  // namespace oqp

// Kernel chosen for an instance: group (a one-wave variant index, or a block
// kernel build after them) and the padded stage sizes of its device records.
struct KSel {
    int group;
    int nx, nu, ng;
};
int group_count();
int select_kernel(const oqp_dims* d, KSel* out);
// km: kernel build (oqp::KM_F64, KM_MIXED, KM_ABS, KM_ROBUST, KM_SOFT)
int group_launch(int g, int km, const oqp::InstDesc* desc, const oqp::InstDesc* hdesc, int count,
                 const double* data, double* iter, double* work, double* step, oqp::DevStat* stat,
                 const oqp::KParams& P, void* stream,
                 bool split_lds = false);
double inst_cost(int N, int nx, int nu);
// kernel build of a solver mode
int kernel_build(int mode);
// stage sizes (dims5: nx, nu, nbu, nbx, ng, each N+1 entries) equal to dims
bool dims5_match(const int* dims5, int N, const oqp_dims* dims);
bool batch_dims_match(const oqp_batch* b, int i, const oqp_dims* dims);
bool server_dims_match(const oqp_server* s, uint64_t ticket, const oqp_dims* dims);

int fail(int code, const char* fmt, ...);
// this device's copy of the library's static device region (scratch.hip):
// its device address and size
int static_dev_region(void** ptr, size_t* bytes);
size_t align_up(size_t v, size_t a);
int check_arg(const oqp_arg* a);
int pick_variant(const oqp_dims* d);
double* qp_field(const oqp_qp* q, int n, int f);
oqp::KParams make_params(const oqp_arg& a, int mode, double tau);
// sslots (may be NULL): device slot of each slack, stage by stage in idxs order
int pack_records(const oqp_qp* q, const oqp::Layout& L, double* dst, int* slots, int* sslots = nullptr);
bool dims_soft(const oqp_dims* d);
void soft_iterate_copy(const int* soft, int N, const oqp::Layout& L, double* rec, bool to_user, double* const vals[6]);
void iterate_user_copy(const int* dims5, int N, const int* slots, const oqp::Layout& L, double* rec, bool to_user,
                       double* u, double* x, double* pi, double* ll, double* lu, double* tl, double* tu);

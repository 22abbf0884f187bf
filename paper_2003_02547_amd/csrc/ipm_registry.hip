// Table of compiled kernel variants (host side).
#include "ipm_launch.h"

namespace oqp {

#define OQP_EXTERN1(x, u, g, km)                                                                                     \
    extern template void launch_ipm<x, u, g, km>(const InstDesc*, int, const double*, double*, double*, double*,    \
                                                 DevStat*, KParams, hipStream_t);
#define OQP_EXTERN(x, u, g) \
    OQP_EXTERN1(x, u, g, KM_F64) OQP_EXTERN1(x, u, g, KM_MIXED) OQP_EXTERN1(x, u, g, KM_ABS) OQP_EXTERN1(x, u, g, KM_ROBUST) \
    OQP_EXTERN1(x, u, g, KM_SOFT) OQP_EXTERN1(x, u, g, KM_BALANCE)
OQP_VARIANTS(OQP_EXTERN)
#undef OQP_EXTERN
#undef OQP_EXTERN1

typedef void (*launch_fn)(const InstDesc*, int, const double*, double*, double*, double*, DevStat*, KParams,
                          hipStream_t);

struct Variant {
    int NX, NU, NG;
    launch_fn fn[6];  // indexed by kernel build (KM_F64, KM_MIXED, KM_ABS, KM_ROBUST, KM_SOFT, KM_BALANCE)
};

#define OQP_ENTRY(x, u, g) \
    {x, u, g,              \
     {&launch_ipm<x, u, g, KM_F64>, &launch_ipm<x, u, g, KM_MIXED>, &launch_ipm<x, u, g, KM_ABS>, &launch_ipm<x, u, g, KM_ROBUST>, \
      &launch_ipm<x, u, g, KM_SOFT>, &launch_ipm<x, u, g, KM_BALANCE>}},
static const Variant kVariants[] = {OQP_VARIANTS(OQP_ENTRY)};
#undef OQP_ENTRY

int variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }

void variant_dims(int v, int* nx, int* nu, int* ng)
{
    *nx = kVariants[v].NX;
    *nu = kVariants[v].NU;
    *ng = kVariants[v].NG;
}

int variant_launch(int v, int km, const InstDesc* desc, int count, const double* data, double* iter, double* work,
                   double* step, DevStat* stat, const KParams& P, void* stream)
{
    if (count <= 0) return 0;
    if (km < KM_F64 || km > KM_BALANCE) return -1;
    kVariants[v].fn[km](desc, count, data, iter, work, step, stat, P, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace oqp

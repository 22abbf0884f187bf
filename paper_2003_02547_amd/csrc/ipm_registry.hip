// Table of compiled kernel variants (host side).
#include "ipm_launch.h"

namespace oqp {

#define OQP_EXTERN(x, u, g)                                                                                           \
    extern template void launch_ipm<x, u, g, false>(const InstDesc*, int, const double*, double*, double*, double*, \
                                                    DevStat*, KParams, hipStream_t);                                 \
    extern template void launch_ipm<x, u, g, true>(const InstDesc*, int, const double*, double*, double*, double*,  \
                                                   DevStat*, KParams, hipStream_t);
OQP_VARIANTS(OQP_EXTERN)
#undef OQP_EXTERN

typedef void (*launch_fn)(const InstDesc*, int, const double*, double*, double*, double*, DevStat*, KParams,
                          hipStream_t);

struct Variant {
    int NX, NU, NG;
    launch_fn fn[2];  // FP64 path, mixed path
};

#define OQP_ENTRY(x, u, g) {x, u, g, {&launch_ipm<x, u, g, false>, &launch_ipm<x, u, g, true>}},
static const Variant kVariants[] = {OQP_VARIANTS(OQP_ENTRY)};
#undef OQP_ENTRY

int variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }

void variant_dims(int v, int* nx, int* nu, int* ng)
{
    *nx = kVariants[v].NX;
    *nu = kVariants[v].NU;
    *ng = kVariants[v].NG;
}

int variant_launch(int v, int mixed, const InstDesc* desc, int count, const double* data, double* iter, double* work,
                   double* step, DevStat* stat, const KParams& P, void* stream)
{
    if (count <= 0) return 0;
    kVariants[v].fn[mixed ? 1 : 0](desc, count, data, iter, work, step, stat, P, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace oqp

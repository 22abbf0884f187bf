// Kernel variants of the batched IPM: compile-time stage sizes (NX, NU, NG)
// covering an instance after padding, each in an FP64 and a mixed build.
#pragma once

#include <hip/hip_runtime.h>

#include "layout.h"

// X(NX, NU, NG) for every compiled variant of the one-wave kernel; the host
// picks the cheapest one that covers an instance.  Larger stage blocks go to
// the runtime-sized block kernel.
#define OQP_VARIANTS(X) \
    X(4, 4, 0) \
    X(4, 4, 4) \
    X(8, 4, 0) \
    X(8, 8, 0) \
    X(8, 16, 0) \
    X(16, 4, 0) \
    X(16, 8, 0) \
    X(16, 16, 0) \
    X(24, 8, 0)

namespace oqp {

template <int NX, int NU, int NG, int KM>
void launch_ipm(const InstDesc* desc, int count, const double* data, double* iter, double* work, double* step,
                DevStat* stat, KParams P, hipStream_t stream);

// block kernel (runtime stage sizes, 256 threads per instance)
int block_lds_bytes(int nx, int nu, int ng);
int block_zmax(int nz);  // compile-time bound used for a stage block of nz (0: too large)
// general rows: kernels for ng == 0 and for 0 < ng <= 64
int block_launch(int zm, int gm, int km, const InstDesc* desc, int count, const double* data, double* iter,
                 double* work, double* step, DevStat* stat, const KParams& P, size_t lds_bytes, void* stream);
// the array-algorithm builds (km == KM_ROBUST, KM_BALANCE), compiled in a unit of their own
int block_launch_qr(int zm, int gm, int km, const InstDesc* desc, int count, const double* data, double* iter,
                    double* work, double* step, DevStat* stat, const KParams& P, size_t lds_bytes, void* stream);
// the soft-constraint build (km == KM_SOFT), compiled in a unit of its own
int block_launch_soft(int zm, int gm, const InstDesc* desc, int count, const double* data, double* iter,
                      double* work, double* step, DevStat* stat, const KParams& P, size_t lds_bytes, void* stream);

// wide-stage kernel (FP64 solve and Newton step; any stage sizes, one
// workgroup per instance, stage matrices in the workspace records)
int wide_lds_bytes(int nx, int nu, int ng);
int wide_launch(const InstDesc* desc, int count, const double* data, double* iter, double* work, double* step,
                DevStat* stat, const KParams& P, size_t lds_bytes, void* stream);

}  // namespace oqp

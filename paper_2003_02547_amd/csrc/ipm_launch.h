// Kernel variants of the batched IPM: compile-time stage sizes (NX, NU, NG)
// covering an instance after padding, each in an FP64 and a mixed build.
#pragma once

#include <hip/hip_runtime.h>

#include "layout.h"

// X(NX, NU, NG) for every compiled variant; the host picks the cheapest one
// that covers an instance.
#define OQP_VARIANTS(X) \
    X(4, 4, 0)          \
    X(4, 4, 4)          \
    X(8, 4, 0)          \
    X(8, 8, 0)          \
    X(8, 16, 0)         \
    X(16, 4, 0)         \
    X(16, 8, 0)         \
    X(16, 16, 0)        \
    X(24, 4, 0)         \
    X(24, 8, 0)         \
    X(24, 16, 0)        \
    X(32, 4, 0)         \
    X(32, 8, 0)         \
    X(32, 16, 0)        \
    X(40, 8, 0)         \
    X(40, 16, 0)        \
    X(48, 8, 0)         \
    X(48, 16, 0)

namespace oqp {

template <int NX, int NU, int NG, bool MIXED>
void launch_ipm(const InstDesc* desc, int count, const double* data, double* iter, double* work, double* step,
                DevStat* stat, KParams P, hipStream_t stream);

}  // namespace oqp

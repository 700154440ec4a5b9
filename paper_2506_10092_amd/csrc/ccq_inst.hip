// Instances of the persistent kernels for one bound on RLE columns.  This
// file is compiled once per (bound, kernel) pair with -DCCQ_KMAX=2|4|8 and
// -DCCQ_BATCH=0|1, so the instances build in parallel.
#include "ccq_device.h"

#ifndef CCQ_KMAX
#error "CCQ_KMAX must be defined"
#endif

#define CCQ_CAT2(a, b) a##b
#define CCQ_CAT(a, b) CCQ_CAT2(a, b)

namespace ccq {

#if CCQ_BATCH
BatchFn CCQ_CAT(batch_kernel_k, CCQ_KMAX)(int w0, bool big) {
    if (w0 == 14) return big ? &k_batch<CCQ_KMAX, 14, true> : &k_batch<CCQ_KMAX, 14, false>;
    if (w0 == 20) return big ? &k_batch<CCQ_KMAX, 20, true> : &k_batch<CCQ_KMAX, 20, false>;
    if (w0 == -1) return &k_batch<CCQ_KMAX, -1, false>;   // staged paths, full instance
    if (w0 == -2) return &k_batch<CCQ_KMAX, -2, false>;   // generic row path, common instance
    return &k_batch<CCQ_KMAX, 0, false>;
}
#else
FusedFn CCQ_CAT(fused_kernel_k, CCQ_KMAX)(int w0, bool big) {
    if (w0 == 14) return big ? &k_fused<CCQ_KMAX, 14, true> : &k_fused<CCQ_KMAX, 14, false>;
    if (w0 == 20) return big ? &k_fused<CCQ_KMAX, 20, true> : &k_fused<CCQ_KMAX, 20, false>;
    if (w0 == -1) return &k_fused<CCQ_KMAX, -1, false>;   // staged paths, full instance
    if (w0 == -2) return &k_fused<CCQ_KMAX, -2, false>;   // generic row path, common instance
    return &k_fused<CCQ_KMAX, 0, false>;
}
#endif

}  // namespace ccq

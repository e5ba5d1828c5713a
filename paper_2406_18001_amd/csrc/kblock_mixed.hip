// Mixed-precision kernel block (placeholder until the MFMA kernels land).
#include "common.hpp"

namespace kdcd {

int64_t kblock_mixed_row_groups(int64_t m, int32_t sb)
{
    (void)m;
    (void)sb;
    return 1;
}

hipError_t launch_kblock_mixed(const KBlockArgs &a, hipStream_t st)
{
    (void)a;
    (void)st;
    return hipErrorNotSupported;
}

hipError_t launch_convert_lowp(const kdcd_matrix *A, int32_t compute, void *hi, void *lo,
                               int64_t ldlow, float *normlow, hipStream_t st)
{
    (void)A; (void)compute; (void)hi; (void)lo; (void)ldlow; (void)normlow; (void)st;
    return hipErrorNotSupported;
}

}  // namespace kdcd

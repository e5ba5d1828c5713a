// CSR kernel block (placeholder until the sparse kernel lands).
#include "common.hpp"

namespace kdcd {

int64_t kblock_csr_row_groups(int64_t m, int32_t sb)
{
    (void)m;
    (void)sb;
    return 1;
}

hipError_t launch_kblock_csr(const KBlockArgs &a, hipStream_t st)
{
    (void)a;
    (void)st;
    return hipErrorNotSupported;
}

}  // namespace kdcd

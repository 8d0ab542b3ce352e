// Split-precision MFMA path (placeholder until the GEMM-DFT kernels land).
#include "../../include/blocktransform.h"
#include "bt_api_internal.hpp"

namespace bt {
int split_supported(int, int, int) { return TF_EUNSUPPORTED; }
size_t split_workspace_size(int64_t, int, int, int64_t, int, int) { return 0; }
int split_prepare(int, int, int) { return TF_EUNSUPPORTED; }
int split_run(int, const void *, const float *, void *, int64_t, int, int, int64_t, int, void *, size_t,
              void *)
{
    return TF_EUNSUPPORTED;
}
} // namespace bt

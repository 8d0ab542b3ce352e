// Ragged batches (placeholder until the persistent kernel lands).
#include "../../include/blocktransform.h"
#include "bt_api_internal.hpp"

extern "C" int transform_ragged_plan_create(const int32_t *, const int32_t *, const int64_t *,
                                            const int64_t *, int64_t, int64_t, tf_ragged_plan *plan)
{
    if (plan) *plan = nullptr;
    return TF_EUNSUPPORTED;
}
extern "C" int transform_ragged_plan_destroy(tf_ragged_plan) { return TF_OK; }
extern "C" int transform_ragged_execute(tf_ragged_plan, int32_t, const void *, const float *, void *,
                                        const void *, float *, int32_t *, int32_t, void *)
{
    return TF_EUNSUPPORTED;
}

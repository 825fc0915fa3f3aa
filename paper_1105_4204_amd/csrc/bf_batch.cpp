// Batched persistent launch (placeholder until the batch kernel lands).
#include "bf_internal.h"

using namespace bf;

struct bf_batch_plan {
    int n;
};

extern "C" {

bf_status bf_batch_plan_create(const bf_image_desc*, int32_t, bf_batch_plan** plan) {
    if (plan) *plan = nullptr;
    set_error("batch plans not implemented yet");
    return BF_EUNSUPPORTED;
}

bf_status bf_batch_bind(bf_batch_plan*, const float* const*, const float* const*, float* const*,
                        float* const*, float* const*, float*) {
    set_error("batch plans not implemented yet");
    return BF_EUNSUPPORTED;
}

bf_status bf_batch_launch(bf_batch_plan*, void*) {
    set_error("batch plans not implemented yet");
    return BF_EUNSUPPORTED;
}

void bf_batch_plan_destroy(bf_batch_plan* plan) { delete plan; }

}  // extern "C"

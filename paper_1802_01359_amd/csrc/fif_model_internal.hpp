// Calls between the plan runtime and the proposal-network runtime (two
// translation units of libfif).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/fif.h"

namespace fif {

// Stores msg as this thread's fif_last_error() message and returns st.
fif_status fif_internal_fail(fif_status st, const std::string& msg);

int32_t model_max_batch(const fif_model* m);
int model_device(const fif_model* m);
// Network outputs of B input rows (B <= model_max_batch), enqueued on s;
// returns the model's device buffer of B x 2 outputs.
const float* model_infer(fif_model* m, const uint16_t* feats, int32_t B, hipStream_t s);

}  // namespace fif

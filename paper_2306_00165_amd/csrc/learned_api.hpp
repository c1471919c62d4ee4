// Internal entry points shared between the C-ABI files.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/pcfv.h"

namespace pcfv {

// MLP forward pass of B rows on an explicit stream (see pcfv_mlp_forward).
pcfv_status mlp_forward_on(pcfv_mlp* mlp, hipStream_t s, const float* X, float* Y, int B);
// Input width, output width and largest batch of an MLP.
void mlp_shape(const pcfv_mlp* mlp, int* din, int* dout, int* max_batch);
// Message returned by pcfv_last_error(NULL) on the calling thread.
void set_create_error(const std::string& msg);

}  // namespace pcfv

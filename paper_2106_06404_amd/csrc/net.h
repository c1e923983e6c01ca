// Internal interface of the warm-start network used by the setup (msdd.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include "msdd.h"

namespace msdd_net_internal {
int n_in(const msdd_net* net);
int n_hidden(const msdd_net* net);
int n_vec(const msdd_net* net);
int n_pos(const msdd_net* net);
int device(const msdd_net* net);
// BF16 inference of `batch` samples, x (batch x n_in) and y (batch x n_vec*n_pos) device
// FP32 arrays, launched on stream s; throws msdd_host::MsddError.
void infer(msdd_net* net, int batch, const float* x, float* y, hipStream_t s);
}  // namespace msdd_net_internal

// unet.h -- host interface of the warm-start network (unet.hip).
#pragma once

#include <cstdint>

#include "internal.h"

namespace ts {

// Number of FP32 parameters (convolution weights [27][Cout][Cin] + biases per
// layer, then the head's 16 weights and bias).
int64_t unet_param_count();

// out[v] = network(input)[v]; input [V][2] FP32 (normalised field, signal
// mask), channels-last; D, H, W multiples of 4.  Device pointers.
void unet_forward(ts_ctx* ctx, const float* params, const float* input, int D, int H, int W,
                  float* out);

// Forward, mean squared error against target [V], and the gradient of that
// loss with respect to every parameter (grad overwritten).  Returns the loss.
double unet_backward(ts_ctx* ctx, const float* params, const float* input, const float* target,
                     int D, int H, int W, float* grad);

// One Adam step (step counts from 1).
void unet_adam(ts_ctx* ctx, float* params, const float* grad, float* m, float* v, int64_t n,
               int64_t step, float lr, float b1, float b2, float eps);

}  // namespace ts

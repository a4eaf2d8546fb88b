// Element-wise precision conversions; see convert.hip.
#pragma once

#include "common.hpp"

namespace apw {

int convert_f64_to_f32(int64_t n, const double *in, float *out, hipStream_t st);
int convert_f32_to_f64(int64_t n, const float *in, double *out, hipStream_t st);

}  // namespace apw

// Element-wise precision conversions and small vector kernels shared by the
// entry points (down-cast copies of V and beta, complex128 <-> complex64).
#include "common.hpp"
#include "convert.hpp"

namespace apw {

template <typename TO, typename TI>
__global__ void k_convert(int64_t n, const TI *__restrict__ in, TO *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = static_cast<TO>(in[i]);
}

static dim3 grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

int convert_f64_to_f32(int64_t n, const double *in, float *out, hipStream_t st) {
    KernelTimer kt("convert", st);
    hipLaunchKernelGGL((k_convert<float, double>), grid_for(n), dim3(256), 0, st, n, in, out);
    return check_launch("convert");
}

int convert_f32_to_f64(int64_t n, const float *in, double *out, hipStream_t st) {
    KernelTimer kt("convert", st);
    hipLaunchKernelGGL((k_convert<double, float>), grid_for(n), dim3(256), 0, st, n, in, out);
    return check_launch("convert");
}

}  // namespace apw

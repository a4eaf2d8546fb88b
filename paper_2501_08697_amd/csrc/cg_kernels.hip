// Kernels of the band-by-band preconditioned conjugate-gradient eigensolver
// (the CG figure of Sec. III.B): vector updates, inner products, and the
// scalar steps (Polak-Ribiere gamma, projection coefficient, normalisation,
// the line-minimising rotation) evaluated on the device from inner products
// left in device memory by the previous launch. Inner products reduce in a
// fixed order in one work-group, so a run repeats bit for bit.
#include <cmath>

#include "cg_kernels.hpp"

namespace apw {

constexpr int kDotThreads = 1024;

__global__ __launch_bounds__(256) void k_cg_axpby(int n, const z64 *__restrict__ a, const z64 *u, const z64 *__restrict__ b,
                                                  const z64 *v, z64 *out) {
    const z64 ca = *a, cb = *b;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const z64 x = u[i], y = v[i];
        out[i] = cmul(ca, x) + cmul(cb, y);
    }
}

// block y = 0: <u1|v1> -> out1; block y = 1: <u2|v2> -> out2
__global__ __launch_bounds__(kDotThreads) void k_cg_dots(int n, const z64 *__restrict__ u1, const z64 *__restrict__ v1,
                                                         double *out1, const z64 *__restrict__ u2,
                                                         const z64 *__restrict__ v2, double *out2, int re_only) {
    __shared__ double red[2][kDotThreads / 64];
    const z64 *u = blockIdx.x == 0 ? u1 : u2;
    const z64 *v = blockIdx.x == 0 ? v1 : v2;
    double *out = blockIdx.x == 0 ? out1 : out2;
    double sr = 0.0, si = 0.0;
    for (int i = threadIdx.x; i < n; i += kDotThreads) {
        const z64 c = cmulc(v[i], u[i]);   // conj(u) v
        sr += c.re;
        si += c.im;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sr += __shfl_xor(sr, o, 64);
        si += __shfl_xor(si, o, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][w] = sr;
        red[1][w] = si;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < kDotThreads / 64; ++q) {
            a += red[0][q];
            b += red[1][q];
        }
        out[0] = a;
        if (!re_only) out[1] = b;
    }
}

// d = 1 * g + gamma * d, gamma = max(0, (gr - grp) / gr_prev), 0 at the first step
__global__ void k_cg_direction(CgScalars *s, int first) {
    const double gamma = first ? 0.0 : fmax(0.0, (s->gr - s->grp) / s->gr_prev);
    s->a1 = z64{1.0, 0.0};
    s->b1 = z64{gamma, 0.0};
    s->gr_prev = s->gr;
}

// d_perp = d - <psi|d> psi
__global__ void k_cg_project(CgScalars *s) {
    s->a1 = z64{1.0, 0.0};
    s->b1 = z64{-s->xd.re, -s->xd.im};
}

// d_hat = d_perp / ||d_perp||
__global__ void k_cg_normalise(CgScalars *s) {
    s->a1 = z64{1.0 / sqrt(s->dn2), 0.0};
    s->b1 = z64{0.0, 0.0};
}

// psi / sqrt(<psi|psi>) (kept in rn2 by the preceding inner product)
__global__ void k_cg_scale_self(CgScalars *s) {
    s->a1 = z64{1.0 / sqrt(s->rn2), 0.0};
    s->b1 = z64{0.0, 0.0};
}

// theta minimises the Rayleigh quotient on span{psi, d_hat}:
// E(theta) = lam cos^2 + 2 b sin cos + c sin^2  ->  theta = atan2(-2b, c - lam) / 2
__global__ void k_cg_rotate(CgScalars *s) {
    const double th = 0.5 * atan2(-2.0 * s->b, s->c - s->lam);
    const double ct = cos(th), sn = sin(th);
    s->a1 = z64{ct, 0.0};
    s->b1 = z64{sn, 0.0};
}

__global__ __launch_bounds__(256) void k_cg_zero(int n, z64 *x) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] = z64{0.0, 0.0};
}

static dim3 grid_for(int n) { return dim3((unsigned)std::min(1024, std::max(1, ceil_div(n, 256)))); }

int cg_axpby(int n, const z64 *a, const z64 *u, const z64 *b, const z64 *v, z64 *out, hipStream_t st) {
    KernelTimer kt("cg_axpby", st);
    hipLaunchKernelGGL(k_cg_axpby, grid_for(n), dim3(256), 0, st, n, a, u, b, v, out);
    return check_launch("cg_axpby");
}

int cg_dots(int n, const z64 *u1, const z64 *v1, double *out1, const z64 *u2, const z64 *v2, double *out2,
            bool re_only, hipStream_t st) {
    KernelTimer kt("cg_dots", st);
    hipLaunchKernelGGL(k_cg_dots, dim3(u2 ? 2 : 1), dim3(kDotThreads), 0, st, n, u1, v1, out1, u2, v2, out2,
                       re_only ? 1 : 0);
    return check_launch("cg_dots");
}

int cg_stage_direction(CgScalars *s, int first, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_direction, dim3(1), dim3(1), 0, st, s, first);
    return check_launch("cg_direction");
}
int cg_stage_project(CgScalars *s, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_project, dim3(1), dim3(1), 0, st, s);
    return check_launch("cg_project");
}
int cg_stage_normalise(CgScalars *s, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_normalise, dim3(1), dim3(1), 0, st, s);
    return check_launch("cg_normalise");
}
int cg_stage_rotate(CgScalars *s, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_rotate, dim3(1), dim3(1), 0, st, s);
    return check_launch("cg_rotate");
}
int cg_stage_scale_self(CgScalars *s, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_scale_self, dim3(1), dim3(1), 0, st, s);
    return check_launch("cg_scale_self");
}
int cg_zero(int n, z64 *x, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_zero, grid_for(n), dim3(256), 0, st, n, x);
    return check_launch("cg_zero");
}

}  // namespace apw

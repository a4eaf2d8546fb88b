// Element-wise and per-band kernels of the block Davidson iteration (Sec.
// III.B names Davidson; the preconditioner is the Teter-Payne-Allan form the
// paper cites for its conjugate-gradient solver). Reductions over G run in a
// fixed order inside one work-group per band, so results repeat bit for bit.
#include "common.hpp"
#include "davidson_kernels.hpp"

namespace apw {

template <int NT> __device__ double wg_sum(double v, double *red) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    __syncthreads();
    return s;
}

// R_n = W_n - lam_n X_n;  rn2[n] = ||R_n||^2;  ek[n] = sum_G |k+G|^2 |X_n(G)|^2.
__global__ __launch_bounds__(256) void k_resid(int npw, const z64 *__restrict__ X, const z64 *__restrict__ W,
                                               const double *__restrict__ lam, const double *__restrict__ kin,
                                               z64 *__restrict__ R, double *__restrict__ rn2, double *__restrict__ ek) {
    __shared__ double red[4];
    const int n = blockIdx.x;
    const z64 *x = X + (int64_t)n * npw;
    const z64 *w = W + (int64_t)n * npw;
    z64 *r = R + (int64_t)n * npw;
    const double l = lam[n];
    double a = 0.0, b = 0.0;
    for (int g = threadIdx.x; g < npw; g += 256) {
        const z64 xv = x[g], wv = w[g];
        const z64 rv = z64{wv.re - l * xv.re, wv.im - l * xv.im};
        r[g] = rv;
        a += rv.re * rv.re + rv.im * rv.im;
        b += kin[g] * (xv.re * xv.re + xv.im * xv.im);
    }
    a = wg_sum<256>(a, red);
    b = wg_sum<256>(b, red);
    if (threadIdx.x == 0) {
        rn2[n] = a;
        ek[n] = b;
    }
}

// T_i = K(x) R_{act[i]},  x = |k+G|^2 / max(ek[act[i]], 1e-3),
// K(x) = (27 + 18x + 12x^2 + 8x^3) / (27 + 18x + 12x^2 + 8x^3 + 16x^4).
__global__ void k_precond(int npw, const int *__restrict__ act, const z64 *__restrict__ R,
                          const double *__restrict__ kin, const double *__restrict__ ek, z64 *__restrict__ T) {
    const int i = blockIdx.y, band = act[i];
    const double inv = 1.0 / fmax(ek[band], 1e-3);
    const z64 *r = R + (int64_t)band * npw;
    z64 *t = T + (int64_t)i * npw;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < npw; g += gridDim.x * blockDim.x) {
        const double x = kin[g] * inv;
        const double num = 27.0 + x * (18.0 + x * (12.0 + 8.0 * x));
        const double k = num / (num + 16.0 * x * x * x * x);
        t[g] = z64{k * r[g].re, k * r[g].im};
    }
}

// out[i] = ||T_i||^2
__global__ __launch_bounds__(256) void k_row_norm2(int npw, const z64 *__restrict__ T, double *__restrict__ out) {
    __shared__ double red[4];
    const z64 *t = T + (int64_t)blockIdx.x * npw;
    double a = 0.0;
    for (int g = threadIdx.x; g < npw; g += 256) a += t[g].re * t[g].re + t[g].im * t[g].im;
    a = wg_sum<256>(a, red);
    if (threadIdx.x == 0) out[blockIdx.x] = a;
}

// dst_i = src_{idx[i]}
__global__ void k_gather_rows(int npw, const int *__restrict__ idx, const z64 *__restrict__ src, z64 *__restrict__ dst) {
    const z64 *s = src + (int64_t)idx[blockIdx.y] * npw;
    z64 *d = dst + (int64_t)blockIdx.y * npw;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < npw; g += gridDim.x * blockDim.x) d[g] = s[g];
}

// New columns of the subspace matrix. C[j*ldc + i] = <v_i | H t_j> for
// i < nb0 + m, j < m (t_j = v_{nb0+j}). Hs is row-major, Hs[i][j] = <v_i|H v_j>.
__global__ void k_hs_append(int nb0, int m, const z64 *__restrict__ C, int ldc, z64 *__restrict__ Hs, int ld) {
    const int n = nb0 + m;
    const int64_t tot = (int64_t)n * m;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(q / n), i = (int)(q - (int64_t)j * n);
        const z64 c = C[(int64_t)j * ldc + i];
        if (i < nb0) {
            Hs[(int64_t)i * ld + nb0 + j] = c;
            Hs[(int64_t)(nb0 + j) * ld + i] = z64{c.re, -c.im};
        } else {
            const int a = i - nb0;
            const z64 o = C[(int64_t)a * ldc + nb0 + j];   // <t_j | H t_a>
            Hs[(int64_t)(nb0 + a) * ld + nb0 + j] = z64{0.5 * (c.re + o.re), 0.5 * (c.im - o.im)};
        }
    }
}

// Hs[0:n, 0:n] = diag(theta)
__global__ void k_hs_diag(int n, const double *__restrict__ theta, z64 *__restrict__ Hs, int ld) {
    const int64_t tot = (int64_t)n * n;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q / n), j = (int)(q - (int64_t)i * n);
        Hs[(int64_t)i * ld + j] = z64{i == j ? theta[i] : 0.0, 0.0};
    }
}

// dst[0:n, 0:n] = src[0:n, 0:n]  (row-major, leading dimensions lds, ldd)
__global__ void k_copy_block(int n, const z64 *__restrict__ src, int lds, z64 *__restrict__ dst, int ldd) {
    const int64_t tot = (int64_t)n * n;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q / n), j = (int)(q - (int64_t)i * n);
        dst[(int64_t)i * ldd + j] = src[(int64_t)i * lds + j];
    }
}

// M = 1.5 I - 0.5 G (first-order Lowdin factor, in place)
__global__ void k_lowdin(int n, z64 *G) {
    const int64_t tot = (int64_t)n * n;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q / n), j = (int)(q - (int64_t)i * n);
        G[q] = z64{(i == j ? 1.5 : 0.0) - 0.5 * G[q].re, -0.5 * G[q].im};
    }
}

// G[i][i] += s
__global__ void k_add_diag(int n, z64 *G, int ld, double s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) G[(int64_t)i * ld + i].re += s;
}

// ------------------------------------------------------------ launchers ----
static dim3 rows_grid(int npw, int m) { return dim3((unsigned)std::min(ceil_div(npw, 256), 64), (unsigned)m); }

int dav_resid(int nb, int npw, const z64 *X, const z64 *W, const double *lam, const double *kin, z64 *R, double *rn2,
              double *ek, hipStream_t st) {
    KernelTimer kt("dav_resid", st);
    hipLaunchKernelGGL(k_resid, dim3(nb), dim3(256), 0, st, npw, X, W, lam, kin, R, rn2, ek);
    return check_launch("dav_resid");
}

int dav_precond(int m, int npw, const int *act, const z64 *R, const double *kin, const double *ek, z64 *T,
                hipStream_t st) {
    KernelTimer kt("dav_precond", st);
    hipLaunchKernelGGL(k_precond, rows_grid(npw, m), dim3(256), 0, st, npw, act, R, kin, ek, T);
    return check_launch("dav_precond");
}

int dav_row_norm2(int m, int npw, const z64 *T, double *out, hipStream_t st) {
    KernelTimer kt("dav_norms", st);
    hipLaunchKernelGGL(k_row_norm2, dim3(m), dim3(256), 0, st, npw, T, out);
    return check_launch("dav_norms");
}

int dav_gather_rows(int m, int npw, const int *idx, const z64 *src, z64 *dst, hipStream_t st) {
    KernelTimer kt("dav_gather", st);
    hipLaunchKernelGGL(k_gather_rows, rows_grid(npw, m), dim3(256), 0, st, npw, idx, src, dst);
    return check_launch("dav_gather");
}

int dav_hs_append(int nb0, int m, const z64 *C, int ldc, z64 *Hs, int ld, hipStream_t st) {
    const int64_t tot = (int64_t)(nb0 + m) * m;
    KernelTimer kt("dav_small", st);
    hipLaunchKernelGGL(k_hs_append, dim3((unsigned)std::min<int64_t>(ceil_div64(tot, 256), 4096)), dim3(256), 0, st,
                       nb0, m, C, ldc, Hs, ld);
    return check_launch("dav_hs_append");
}

int dav_hs_diag(int n, const double *theta, z64 *Hs, int ld, hipStream_t st) {
    KernelTimer kt("dav_small", st);
    hipLaunchKernelGGL(k_hs_diag, dim3((unsigned)std::min<int64_t>(ceil_div64((int64_t)n * n, 256), 4096)),
                       dim3(256), 0, st, n, theta, Hs, ld);
    return check_launch("dav_hs_diag");
}

int dav_copy_block(int n, const z64 *src, int lds, z64 *dst, int ldd, hipStream_t st) {
    KernelTimer kt("dav_small", st);
    hipLaunchKernelGGL(k_copy_block, dim3((unsigned)std::min<int64_t>(ceil_div64((int64_t)n * n, 256), 4096)),
                       dim3(256), 0, st, n, src, lds, dst, ldd);
    return check_launch("dav_copy_block");
}

int dav_lowdin(int n, z64 *G, hipStream_t st) {
    KernelTimer kt("dav_small", st);
    hipLaunchKernelGGL(k_lowdin, dim3((unsigned)std::min<int64_t>(ceil_div64((int64_t)n * n, 256), 1024)), dim3(256), 0,
                       st, n, G);
    return check_launch("dav_lowdin");
}

int dav_add_diag(int n, z64 *G, int ld, double s, hipStream_t st) {
    KernelTimer kt("dav_small", st);
    hipLaunchKernelGGL(k_add_diag, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, G, ld, s);
    return check_launch("dav_add_diag");
}

}  // namespace apw

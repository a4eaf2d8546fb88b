// Small dense FP64 linear algebra on the GPU for the Davidson subspace
// (Sec. III.B names Davidson; its Rayleigh-Ritz and orthonormalisation steps
// need a Cholesky factorisation and a Hermitian eigensolver of the subspace
// matrix, kept in FP64 on the device):
//
//   k_potrf_inv  Cholesky G = L L^H of a Hermitian positive definite matrix and
//                the inverse L^{-1} (one work-group).
//   k_hetrd      Householder reduction of a Hermitian matrix to a real
//                symmetric tridiagonal T = Q^H A Q (one work-group; the
//                reflector convention H = I - tau v v^H, v[0] = 1, makes every
//                off-diagonal real).
//   k_stebz      eigenvalues of T by bisection on Sturm counts; one wavefront per
//                eigenvalue, each of its 64 lanes evaluating one point of a
//                65-way multisection of the current bracket.
//   k_stein      eigenvectors of T by inverse iteration with a pivoted
//                tridiagonal LU; eigenvalues closer than 1e-7 ||T|| form a
//                cluster handled by one thread, which re-orthogonalises the
//                cluster's vectors (modified Gram-Schmidt) after every solve.
//                Between clusters inverse iteration leaves a non-orthogonality
//                of at most eps ||T|| / gap (2e-9); callers remove it with one
//                Lowdin step (see the Davidson driver).
//   k_unmtr      y = Q z for every wanted eigenvector (one work-group each).
//
// All matrices are row-major with a leading dimension.
#include "common.hpp"
#include "dense.hpp"

namespace apw {

constexpr int kNT = 1024;
constexpr double kClusterTol = 1e-7;   // relative eigenvalue gap below which vectors are orthogonalised together

__device__ __forceinline__ z64 zconj(z64 a) { return z64{a.re, -a.im}; }
__device__ __forceinline__ double zabs2(z64 a) { return a.re * a.re + a.im * a.im; }

// Block-wide sum of one double per thread (fixed order: deterministic).
__device__ double block_sum(double v, double *red) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    __syncthreads();
    return s;
}

// --------------------------------------------------------------- Cholesky --
// G (n x n, ld) Hermitian positive definite; its lower triangle is replaced
// by L with G = L L^H. Linv (n x n, ldi) receives L^{-1} (zero above the
// diagonal). info = 0, or k + 1 when the k-th pivot is not positive.
__global__ __launch_bounds__(kNT) void k_potrf_inv(int n, z64 *G, int ld, z64 *Linv, int ldi, int *info) {
    const int tid = threadIdx.x;
    for (int k = 0; k < n; ++k) {
        __syncthreads();
        const double dkk = G[(int64_t)k * ld + k].re;
        if (!(dkk > 0.0) || !isfinite(dkk)) {
            if (tid == 0) *info = k + 1;
            return;
        }
        const double lkk = sqrt(dkk), inv = 1.0 / lkk;
        for (int i = k + 1 + tid; i < n; i += kNT) {
            z64 &g = G[(int64_t)i * ld + k];
            g = z64{g.re * inv, g.im * inv};
        }
        __syncthreads();
        if (tid == 0) G[(int64_t)k * ld + k] = z64{lkk, 0.0};
        const int m = n - k - 1;
        for (int idx = tid; idx < m * m; idx += kNT) {
            const int i = idx / m, j = idx - i * m;
            if (j > i) continue;
            const z64 a = G[(int64_t)(k + 1 + i) * ld + k], b = G[(int64_t)(k + 1 + j) * ld + k];
            z64 &g = G[(int64_t)(k + 1 + i) * ld + k + 1 + j];
            g = g - cmulc(a, b);
        }
    }
    __syncthreads();
    if (tid == 0) *info = 0;
    // forward substitution, one column c of L^{-1} per thread
    for (int c = tid; c < n; c += kNT) {
        for (int i = 0; i < c; ++i) Linv[(int64_t)i * ldi + c] = z64{0.0, 0.0};
        for (int i = c; i < n; ++i) {
            z64 s = z64{i == c ? 1.0 : 0.0, 0.0};
            for (int q = c; q < i; ++q) s = s - cmul(G[(int64_t)i * ld + q], Linv[(int64_t)q * ldi + c]);
            const double lii = G[(int64_t)i * ld + i].re;
            Linv[(int64_t)i * ldi + c] = z64{s.re / lii, s.im / lii};
        }
    }
}

// ------------------------------------------------------------- tridiagonal --
// A (n x n, ld) Hermitian, full storage. On exit d[n], e[n-1] hold T and
// column k of A below row k+1 holds v_k (v_k[k+1] = 1 implicit), tau[k] its
// factor, so Q = H_0 H_1 ... H_{n-2}.
__global__ __launch_bounds__(kNT) void k_hetrd(int n, z64 *A, int ld, double *d, double *e, z64 *tau) {
    __shared__ z64 v[kMaxSub];
    __shared__ z64 y[kMaxSub];
    __shared__ z64 part[kNT];
    __shared__ double red[kNT / 64];
    const int tid = threadIdx.x;
    for (int k = 0; k < n - 1; ++k) {
        const int m = n - k - 1;
        z64 *col = A + (int64_t)(k + 1) * ld + k;
        const z64 alpha = col[0];   // read before the barriers of block_sum: col[0] is rewritten below
        double p = 0.0;
        for (int i = 1 + tid; i < m; i += kNT) p += zabs2(col[(int64_t)i * ld]);
        const double xn2 = block_sum(p, red);
        z64 t = z64{0.0, 0.0};
        double beta = alpha.re;
        z64 scale = z64{0.0, 0.0};
        if (!(xn2 == 0.0 && alpha.im == 0.0)) {
            beta = -copysign(sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn2), alpha.re);
            t = z64{(beta - alpha.re) / beta, -alpha.im / beta};
            const z64 den = z64{alpha.re - beta, alpha.im};     // scale = 1 / (alpha - beta)
            const double dd = zabs2(den);
            scale = z64{den.re / dd, -den.im / dd};
        }
        if (tid == 0) {
            d[k] = A[(int64_t)k * ld + k].re;
            e[k] = beta;
            tau[k] = t;
        }
        if (t.re == 0.0 && t.im == 0.0) {
            if (tid == 0) col[0] = z64{1.0, 0.0};
            continue;
        }
        for (int i = tid; i < m; i += kNT) {
            z64 vi = i == 0 ? z64{1.0, 0.0} : cmul(col[(int64_t)i * ld], scale);
            v[i] = vi;
            col[(int64_t)i * ld] = vi;
        }
        __syncthreads();
        // y = tau * A22 v with A22[i][j] = conj(A22[j][i]): lanes run along a row for coalescing
        const int mp = (m + 63) / 64 * 64;      // m < kMaxSub <= kNT
        const int G = kNT / mp;
        z64 *A22 = A + (int64_t)(k + 1) * ld + k + 1;
        {
            const int i = tid % mp, g = tid / mp;
            z64 acc = z64{0.0, 0.0};
            if (g < G && i < m)
                for (int j = g; j < m; j += G) acc = acc + cmul(zconj(A22[(int64_t)j * ld + i]), v[j]);
            part[tid] = acc;
            __syncthreads();
            if (tid < m) {
                z64 s = z64{0.0, 0.0};
                for (int q = 0; q < G; ++q) s = s + part[q * mp + tid];
                y[tid] = cmul(t, s);
            }
            __syncthreads();
        }
        // alpha2 = -1/2 tau (y^H v); w = y + alpha2 v
        double pr = 0.0, pi = 0.0;
        for (int i = tid; i < m; i += kNT) {
            const z64 c = cmulc(v[i], y[i]);     // conj(y) v
            pr += c.re;
            pi += c.im;
        }
        const double sr = block_sum(pr, red), si = block_sum(pi, red);
        const z64 a2 = cmul(z64{-0.5 * t.re, -0.5 * t.im}, z64{sr, si});
        for (int i = tid; i < m; i += kNT) y[i] = y[i] + cmul(a2, v[i]);
        __syncthreads();
        // A22 -= v w^H + w v^H
        for (int idx = tid; idx < m * m; idx += kNT) {
            const int i = idx / m, j = idx - i * m;
            z64 &a = A22[(int64_t)i * ld + j];
            a = a - cmulc(v[i], y[j]) - cmulc(y[i], v[j]);
        }
        __syncthreads();
    }
    if (tid == 0) d[n - 1] = A[(int64_t)(n - 1) * ld + n - 1].re;
}

// Number of eigenvalues of T below x (Sturm sequence of the LDL^T pivots).
__device__ __forceinline__ int sturm_count(int n, const double *d, const double *e2, double x, double pivmin) {
    int c = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
    for (int i = 1; i < n; ++i) {
        q = (d[i] - x) - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++c;
    }
    return c;
}

// Eigenvalues j = j0 .. j0+nw-1 (ascending) of T; one wavefront each.
__global__ __launch_bounds__(256) void k_stebz(int n, const double *d, const double *e, int nw, double *w) {
    __shared__ double e2s[kMaxSub];
    __shared__ double ds[kMaxSub];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        ds[i] = d[i];
        e2s[i] = i < n - 1 ? e[i] * e[i] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (j >= nw) return;
    double lo = ds[0], hi = ds[0], emax = 0.0, anorm = 0.0;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0);
        lo = fmin(lo, ds[i] - r);
        hi = fmax(hi, ds[i] + r);
        emax = fmax(emax, i < n - 1 ? e2s[i] : 0.0);
        anorm = fmax(anorm, fabs(ds[i]) + r);
    }
    const double eps = 2.220446049250313e-16;
    const double pivmin = fmax(2.2250738585072014e-308 * fmax(emax, 1.0), 1e-300);
    lo -= 4.0 * eps * anorm + 4.0 * pivmin;
    hi += 4.0 * eps * anorm + 4.0 * pivmin;
    const double tol = 2.0 * eps * anorm + 2.0 * pivmin;
    for (int it = 0; it < 64; ++it) {
        if (hi - lo <= fmax(2.0 * eps * fmax(fabs(lo), fabs(hi)), tol)) break;
        const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
        const int c = sturm_count(n, ds, e2s, x, pivmin);
        const unsigned long long above = __ballot(c > j);   // lanes whose point lies above eigenvalue j
        double nlo = lo, nhi = hi;
        if (above == 0ull) {
            nlo = lo + (hi - lo) * 64.0 / 65.0;
        } else {
            const int f = __ffsll((long long)above) - 1;   // first lane above
            nhi = lo + (hi - lo) * (double)(f + 1) / 65.0;
            if (f > 0) nlo = lo + (hi - lo) * (double)f / 65.0;
        }
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0) w[j] = 0.5 * (lo + hi);
}

__device__ __forceinline__ double hash_uniform(unsigned j, unsigned i) {
    unsigned x = j * 0x9E3779B9u ^ (i + 0x7F4A7C15u) * 0x85EBCA6Bu;
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return (double)(x >> 8) * (2.0 / 16777216.0) - 1.0;
}

// Eigenvectors z_j (column j of Z, ldz) of T for the nw lowest eigenvalues w.
// scratch: 5 n doubles per thread slot (nw slots).
__global__ void k_stein(int n, const double *d, const double *e, int nw, const double *w, double *Z, int ldz,
                        double *scratch) {
    const int j0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (j0 >= nw) return;
    double anorm = 0.0;
    for (int i = 0; i < n; ++i)
        anorm = fmax(anorm, fabs(d[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0));
    const double eps = 2.220446049250313e-16;
    const double ortol = kClusterTol * anorm;
    if (j0 > 0 && w[j0] - w[j0 - 1] <= ortol) return;   // not the first of its cluster
    int j1 = j0 + 1;
    while (j1 < nw && w[j1] - w[j1 - 1] <= ortol) ++j1;
    double *dd = scratch + (int64_t)j0 * 5 * n, *dl = dd + n, *du = dl + n, *du2 = du + n, *x = du2 + n;
    const double tiny = eps * fmax(anorm, 1e-300);
    double lam_prev = 0.0;
    for (int j = j0; j < j1; ++j) {
        double lam = w[j];
        if (j > j0 && lam - lam_prev < 10.0 * eps * fmax(fabs(lam), anorm * eps)) lam = lam_prev + 10.0 * eps * fmax(fabs(lam), anorm * eps);
        lam_prev = lam;
        // pivoted LU of T - lam I
        for (int i = 0; i < n; ++i) {
            dd[i] = d[i] - lam;
            if (i < n - 1) {
                dl[i] = e[i];
                du[i] = e[i];
            }
            du2[i] = 0.0;
        }
        unsigned long long pivbits[16] = {0};   // n <= 1024
        for (int i = 0; i < n - 1; ++i) {
            if (fabs(dd[i]) >= fabs(dl[i])) {
                const double den = fabs(dd[i]) < tiny ? copysign(tiny, dd[i] == 0.0 ? 1.0 : dd[i]) : dd[i];
                dd[i] = den;
                const double f = dl[i] / den;
                dl[i] = f;
                dd[i + 1] -= f * du[i];
            } else {
                const double f = dd[i] / dl[i];
                dd[i] = dl[i];
                dl[i] = f;
                const double tmp = du[i];
                du[i] = dd[i + 1];
                dd[i + 1] = tmp - f * dd[i + 1];
                if (i < n - 2) {
                    du2[i] = du[i + 1];
                    du[i + 1] = -f * du[i + 1];
                }
                pivbits[i >> 6] |= 1ull << (i & 63);
            }
        }
        if (fabs(dd[n - 1]) < tiny) dd[n - 1] = copysign(tiny, dd[n - 1] == 0.0 ? 1.0 : dd[n - 1]);
        for (int i = 0; i < n; ++i) x[i] = hash_uniform((unsigned)j, (unsigned)i);
        for (int it = 0; it < 4; ++it) {
            // solve L U x = b in place
            for (int i = 0; i < n - 1; ++i) {
                if (pivbits[i >> 6] & (1ull << (i & 63))) {
                    const double tmp = x[i];
                    x[i] = x[i + 1];
                    x[i + 1] = tmp - dl[i] * x[i];
                } else {
                    x[i + 1] -= dl[i] * x[i];
                }
            }
            x[n - 1] /= dd[n - 1];
            if (n > 1) x[n - 2] = (x[n - 2] - du[n - 2] * x[n - 1]) / dd[n - 2];
            for (int i = n - 3; i >= 0; --i) x[i] = (x[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) / dd[i];
            // re-orthogonalise inside the cluster, then normalise
            for (int q = j0; q < j; ++q) {
                double s = 0.0;
                for (int i = 0; i < n; ++i) s += Z[(int64_t)q * ldz + i] * x[i];
                for (int i = 0; i < n; ++i) x[i] -= s * Z[(int64_t)q * ldz + i];
            }
            double nrm = 0.0;
            for (int i = 0; i < n; ++i) nrm = fmax(nrm, fabs(x[i]));
            for (int i = 0; i < n; ++i) x[i] /= nrm;
            double s2 = 0.0;
            for (int i = 0; i < n; ++i) s2 += x[i] * x[i];
            const double inv = 1.0 / sqrt(s2);
            for (int i = 0; i < n; ++i) x[i] *= inv;
        }
        for (int i = 0; i < n; ++i) Z[(int64_t)j * ldz + i] = x[i];
    }
}

// coef[j*ldc + i] = (Q z_j)[i]: apply H_{n-2} .. H_0 to each real eigenvector.
__global__ __launch_bounds__(256) void k_unmtr(int n, const z64 *A, int ld, const z64 *tau, const double *Z, int ldz,
                                               z64 *coef, int ldc) {
    __shared__ z64 yv[kMaxSub];
    __shared__ double red[4];
    const int j = blockIdx.x, tid = threadIdx.x;
    for (int i = tid; i < n; i += blockDim.x) yv[i] = z64{Z[(int64_t)j * ldz + i], 0.0};
    __syncthreads();
    for (int k = n - 2; k >= 0; --k) {
        const z64 t = tau[k];
        if (t.re == 0.0 && t.im == 0.0) continue;
        // s = v_k^H y over rows k+1 .. n-1 (v_k[k+1] = 1)
        double pr = 0.0, pi = 0.0;
        for (int i = k + 1 + tid; i < n; i += blockDim.x) {
            const z64 vi = i == k + 1 ? z64{1.0, 0.0} : A[(int64_t)i * ld + k];
            const z64 c = cmulc(yv[i], vi);   // conj(v) y
            pr += c.re;
            pi += c.im;
        }
        const double sr = block_sum(pr, red), si = block_sum(pi, red);
        const z64 ts = cmul(t, z64{sr, si});
        for (int i = k + 1 + tid; i < n; i += blockDim.x) {
            const z64 vi = i == k + 1 ? z64{1.0, 0.0} : A[(int64_t)i * ld + k];
            yv[i] = yv[i] - cmul(vi, ts);
        }
        __syncthreads();
    }
    for (int i = tid; i < n; i += blockDim.x) coef[(int64_t)j * ldc + i] = yv[i];
}

// ---------------------------------------------------------------- drivers --
int potrf_inv(int n, z64 *G, int ld, z64 *Linv, int ldi, int *info_dev, hipStream_t st) {
    if (n > kMaxSub) return set_error(ABACUS_PW_EBAD_SHAPE, "Cholesky size above the device limit");
    KernelTimer kt("potrf_inv", st);
    hipLaunchKernelGGL(k_potrf_inv, dim3(1), dim3(kNT), 0, st, n, G, ld, Linv, ldi, info_dev);
    return check_launch("potrf_inv");
}

size_t heev_scratch_bytes(int n) { return (size_t)n * (2 * sizeof(double) + sizeof(z64)) + (size_t)n * n * sizeof(double) * 6 + 1024; }

int heev_lowest(int n, z64 *A, int ld, int nw, double *w, z64 *coef, int ldc, void *scratch, hipStream_t st) {
    if (n > kMaxSub) return set_error(ABACUS_PW_EBAD_SHAPE, "subspace size above the device eigensolver limit");
    char *s = static_cast<char *>(scratch);
    double *d = reinterpret_cast<double *>(s);
    double *e = d + n;
    z64 *tau = reinterpret_cast<z64 *>(e + n);
    double *Z = reinterpret_cast<double *>(tau + n);
    double *work = Z + (size_t)n * n;
    {
        KernelTimer kt("hetrd", st);
        hipLaunchKernelGGL(k_hetrd, dim3(1), dim3(kNT), 0, st, n, A, ld, d, e, tau);
        APW_TRY(check_launch("hetrd"));
    }
    {
        KernelTimer kt("stebz", st);
        hipLaunchKernelGGL(k_stebz, dim3(ceil_div(nw, 4)), dim3(256), 0, st, n, d, e, nw, w);
        APW_TRY(check_launch("stebz"));
    }
    {
        KernelTimer kt("stein", st);
        hipLaunchKernelGGL(k_stein, dim3(ceil_div(nw, 64)), dim3(64), 0, st, n, d, e, nw, w, Z, n, work);
        APW_TRY(check_launch("stein"));
    }
    {
        KernelTimer kt("unmtr", st);
        hipLaunchKernelGGL(k_unmtr, dim3(nw), dim3(256), 0, st, n, A, ld, tau, Z, n, coef, ldc);
        APW_TRY(check_launch("unmtr"));
    }
    return ABACUS_PW_OK;
}

}  // namespace apw

// Dense FP64 linear algebra of the Davidson subspace for orders too large for
// one compute unit (Rayleigh-Ritz over up to ndim * nb basis vectors, Sec. III.B
// Davidson; 2048 for 1024 bands at ndim = 2). The one-CU kernels of dense.hip
// stream the whole trailing matrix through a single CU for every column; here
// every column's matrix-vector product runs over the whole GPU and the O(n^3)
// updates run on the MFMA GEMMs.
//
// Tridiagonal reduction T = Q^H A Q (LAPACK's blocked scheme, restated): columns
// are reduced in panels of kPL. For column k of a panel (c = k - k0):
//   k_trd_col   (one work-group) finishes the previous column's w vector
//               (w = y - tau/2 (y^H v) v), forms column k as stored minus the
//               panel's rank-2 updates so far (A - V W^H - W V^H), builds the
//               Householder reflector H = I - tau v v^H (v[k+1] = 1, real
//               off-diagonal beta) and the dot products W^H v, V^H v;
//   k_trd_hemv  (m / 4 work-groups, one wavefront per row) y = tau (A22 v -
//               V (W^H v) - W (V^H v)) with A22 the trailing matrix as it was
//               when the panel started, read row by row (coalesced, Hermitian
//               full storage).
// After the panel the trailing matrix takes all its updates at once,
// A22 -= [V W] [W V]^H, one complex GEMM with K = 2 kPL on the matrix cores.
//
// Back-transformation coef = Q Z (Z the real tridiagonal eigenvectors): the
// reflectors, kept as rows of Vr, are applied in blocks of kPL from the last to
// the first as I - V T V^H (compact WY; T upper triangular from the block's
// Gram matrix and the taus), each block two GEMMs.
//
// Cholesky G = L L^H in blocks of kCB columns: the diagonal block is factored
// and inverted in LDS by one work-group, the panel below it is L21 = A21 L11^-H
// (GEMM) and the trailing matrix takes A22 -= L21 L21^H (GEMM).
#include <algorithm>

#include "common.hpp"
#include "dense.hpp"
#include "gemm.hpp"

namespace apw {

namespace {

constexpr int kPL = 32;       // columns per panel of the tridiagonal reduction (and reflectors per WY block)
constexpr int kColThreads = 1024;
constexpr int kCB = 64;       // columns per block of the blocked Cholesky

__device__ __forceinline__ z64 zc(z64 a) { return z64{a.re, -a.im}; }
__device__ __forceinline__ double za2(z64 a) { return a.re * a.re + a.im * a.im; }

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the work-group (fixed order).
__device__ double bsum(double v, double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wsum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

// Panel buffers: PX row i = [V[i][0..kPL) | W[i][0..kPL)], PY row i = [W | V].
struct TrdArgs {
    int n, ld;
    z64 *A;
    double *d, *e;
    z64 *tau;
    z64 *Vr;      // [n][n] reflector rows (zero outside k+1 .. n-1)
    z64 *PX, *PY; // [n][2 kPL]
    z64 *PXc;     // [2 kPL][n]: PX by columns, so that reads over rows are coalesced
    z64 *vbuf;    // [n] current reflector, contiguous
    z64 *y;       // [n] tau (A22 v - ...) of the current column
    z64 *s;       // [2 kPL]: W^H v then V^H v
};

// mode 0: finish w of panel column c-1 (if c > 0), then reduce column k = k0 + c.
// mode 1: only finish w of panel column c-1 (end of a panel).
__global__ __launch_bounds__(kColThreads) void k_trd_col(TrdArgs a, int k0, int c, int mode) {
    __shared__ z64 wl[kMaxSub];    // w of panel column c-1, rows k ..
    __shared__ z64 al[kMaxSub];    // column k, rows k ..
    __shared__ double red[kColThreads / 64];
    __shared__ z64 zred[2][kColThreads / 64];
    const int n = a.n, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = kColThreads / 64;
    const int k = k0 + c;   // column to reduce (mode 0); w of column k - 1 is finished first
    if (c > 0) {
        // w = y + alpha v over rows kp + 1 .. n - 1, kp = k - 1, alpha = -tau/2 (y^H v)
        const int kp = k - 1;
        double pr = 0.0, pi = 0.0;
        for (int i = kp + 1 + tid; i < n; i += kColThreads) {
            const z64 yv = a.y[i], v = a.vbuf[i];
            pr += yv.re * v.re + yv.im * v.im;   // conj(y) v
            pi += yv.re * v.im - yv.im * v.re;
        }
        pr = wsum(pr);
        pi = wsum(pi);
        __syncthreads();
        if (lane == 0) {
            zred[0][wv] = z64{pr, 0.0};
            zred[1][wv] = z64{pi, 0.0};
        }
        __syncthreads();
        double sr = 0.0, si = 0.0;
        for (int q = 0; q < nwv; ++q) {
            sr += zred[0][q].re;
            si += zred[1][q].re;
        }
        const z64 t = a.tau[kp];
        const z64 al2 = cmul(z64{-0.5 * t.re, -0.5 * t.im}, z64{sr, si});
        for (int i = kp + 1 + tid; i < n; i += kColThreads) {
            const z64 w = a.y[i] + cmul(al2, a.vbuf[i]);
            wl[i] = w;
            a.PX[(int64_t)i * 2 * kPL + kPL + (c - 1)] = w;
            a.PY[(int64_t)i * 2 * kPL + (c - 1)] = w;
            a.PXc[(int64_t)(kPL + c - 1) * n + i] = w;
        }
        __syncthreads();
    }
    if (mode == 1) return;
    // row k of the panel (V then W), the same for every row below
    __shared__ z64 pk[2 * kPL];
    if (tid < c) {
        pk[tid] = a.PXc[(int64_t)tid * n + k];
        pk[kPL + tid] = tid == c - 1 ? wl[k] : a.PXc[(int64_t)(kPL + tid) * n + k];
    }
    __syncthreads();
    // column k, rows k .. n-1: conj(row k of A) minus the panel's updates of columns q < c
    // (the panel read by columns: consecutive threads, consecutive rows)
    // Eight columns' values are loaded before any is used, so their latencies overlap; the
    // index is clamped to c - 1 (a valid address) and values beyond c are not used. Column
    // c - 1 of W is being written by this kernel: its values come from wl instead.
    for (int i = k + tid; i < n; i += kColThreads) {
        z64 x = zc(a.A[(int64_t)k * a.ld + i]);
        for (int q0 = 0; q0 < c; q0 += 8) {
            z64 vi[8], wi[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = min(q0 + u, c - 1);
                vi[u] = a.PXc[(int64_t)q * n + i];
                wi[u] = a.PXc[(int64_t)(kPL + q) * n + i];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = q0 + u;
                if (q < c) {
                    const z64 w = q == c - 1 ? wl[i] : wi[u];
                    x = x - cmulc(vi[u], pk[kPL + q]) - cmulc(w, pk[q]);   // v_i conj(w_k) + w_i conj(v_k)
                }
            }
        }
        al[i] = x;
    }
    __syncthreads();
    // reflector from x = al[k+1 ..]
    double p = 0.0;
    for (int i = k + 2 + tid; i < n; i += kColThreads) p += za2(al[i]);
    const double xn2 = bsum(p, red);
    const z64 alpha = al[k + 1];
    __syncthreads();   // every thread holds alpha before al[k+1] is overwritten below
    double beta = alpha.re;
    z64 t = z64{0.0, 0.0}, scale = z64{0.0, 0.0};
    if (!(xn2 == 0.0 && alpha.im == 0.0)) {
        beta = -copysign(sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn2), alpha.re);
        t = z64{(beta - alpha.re) / beta, -alpha.im / beta};
        const z64 den = z64{alpha.re - beta, alpha.im};
        const double dd = za2(den);
        scale = z64{den.re / dd, -den.im / dd};
    }
    if (tid == 0) {
        a.d[k] = al[k].re;
        a.e[k] = beta;
        a.tau[k] = t;
    }
    for (int i = tid; i < n; i += kColThreads) {
        z64 v = z64{0.0, 0.0};
        if (i == k + 1) v = z64{1.0, 0.0};
        else if (i > k + 1) v = cmul(al[i], scale);
        a.Vr[(int64_t)k * n + i] = v;
        if (i > k) {
            a.vbuf[i] = v;
            al[i] = v;   // al now holds v
            a.PX[(int64_t)i * 2 * kPL + c] = v;
            a.PY[(int64_t)i * 2 * kPL + kPL + c] = v;
            a.PXc[(int64_t)c * n + i] = v;
        }
    }
    __syncthreads();
    // W^H v and V^H v over rows k+1 .. for the panel columns q < c (one wave per dot product)
    for (int q2 = wv; q2 < 2 * c; q2 += nwv) {
        const bool isw = q2 < c;
        const int q = isw ? q2 : q2 - c;
        const bool from_wl = isw && q == c - 1;   // the W column this kernel wrote
        const z64 *col = a.PXc + (int64_t)(isw ? kPL + q : q) * n;
        double sr = 0.0, si = 0.0;
        int i = k + 1 + lane;
        for (; i + 192 < n; i += 256) {   // four rows per lane in flight
            z64 u[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) u[r] = from_wl ? wl[i + 64 * r] : col[i + 64 * r];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const z64 pr = cmulc(al[i + 64 * r], u[r]);   // conj(u) v
                sr += pr.re;
                si += pr.im;
            }
        }
        for (; i < n; i += 64) {
            const z64 u = from_wl ? wl[i] : col[i];
            const z64 pr = cmulc(al[i], u);
            sr += pr.re;
            si += pr.im;
        }
        sr = wsum(sr);
        si = wsum(si);
        if (lane == 0) a.s[(isw ? 0 : kPL) + q] = z64{sr, si};
    }
}

// y[i] = tau (sum_j A[i][j] v[j] - sum_q V[i][q] s_w[q] - W[i][q] s_v[q]) for rows i > k, j > k.
// v is staged in LDS (dynamic, (n - k - 1) values, vl[j - k - 1] = v[j]).
__global__ __launch_bounds__(256) void k_trd_hemv(TrdArgs a, int k, int c) {
    extern __shared__ __align__(16) unsigned char smem_hemv[];
    z64 *vl = reinterpret_cast<z64 *>(smem_hemv) - (k + 1);
    const int n = a.n, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int j = k + 1 + threadIdx.x; j < n; j += blockDim.x) vl[j] = a.vbuf[j];
    __syncthreads();
    const int i = k + 1 + blockIdx.x * 4 + wv;
    if (i >= n) return;
    const z64 *row = a.A + (int64_t)i * a.ld;
    double sr = 0.0, si = 0.0;
    int j = k + 1 + lane;
    for (; j + 192 < n; j += 256) {
        z64 r[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = row[j + 64 * u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const z64 pr = cmul(r[u], vl[j + 64 * u]);
            sr += pr.re;
            si += pr.im;
        }
    }
    for (; j < n; j += 64) {
        const z64 pr = cmul(row[j], vl[j]);
        sr += pr.re;
        si += pr.im;
    }
    // panel corrections: lane q < c takes V[i][q] s_w[q] + W[i][q] s_v[q]
    if (lane < c) {
        const z64 *px = a.PX + (int64_t)i * 2 * kPL;
        const z64 cr = cmul(px[lane], a.s[lane]) + cmul(px[kPL + lane], a.s[kPL + lane]);
        sr -= cr.re;
        si -= cr.im;
    }
    sr = wsum(sr);
    si = wsum(si);
    if (lane == 0) a.y[i] = cmul(a.tau[k], z64{sr, si});
}

__global__ void k_trd_last(const z64 *A, int ld, int n, double *d) {
    if (threadIdx.x == 0 && blockIdx.x == 0) d[n - 1] = A[(int64_t)(n - 1) * ld + n - 1].re;
}

__global__ void k_zero(z64 *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = z64{0.0, 0.0};
}

// coef[j][i] = Z[j][i] (real eigenvector rows to complex rows of ld ldc)
__global__ void k_real_rows(const double *Z, int ldz, int n, int nw, z64 *coef, int ldc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * nw) return;
    const int j = (int)(t / n), i = (int)(t - (int64_t)j * n);
    coef[(int64_t)j * ldc + i] = z64{Z[(int64_t)j * ldz + i], 0.0};
}

// T (upper triangular, nbk x nbk, row-major) of the compact WY form of H_0 ... H_{nbk-1}:
// T[q][q] = tau_q, T[r][q] = -tau_q sum_{s = r}^{q-1} T[r][s] G[s][q] for r < q, where
// G[s][q] = v_s^H v_q is given transposed: Gt[q * nbk + s] = G[s][q].
__global__ void k_wy_t(int nbk, const z64 *tau, const z64 *Gt, z64 *T) {
    __shared__ z64 Ts[kPL][kPL];
    const int r = threadIdx.x;
    for (int q = 0; q < nbk; ++q) {
        if (r < q) {
            z64 acc = z64{0.0, 0.0};
            for (int s2 = r; s2 < q; ++s2) acc = acc + cmul(Ts[r][s2], Gt[q * nbk + s2]);
            const z64 tq = tau[q];
            Ts[r][q] = z64{-(tq.re * acc.re - tq.im * acc.im), -(tq.re * acc.im + tq.im * acc.re)};
        } else if (r == q) {
            Ts[q][q] = tau[q];
        } else if (r < nbk) {
            Ts[r][q] = z64{0.0, 0.0};
        }
        __syncthreads();
    }
    for (int q = 0; q < nbk; ++q)
        if (r < nbk) T[r * nbk + q] = Ts[r][q];
}

// S'[j][q] = sum_r T[q][r] S[j][r]   (S, S' are [nw][nbk])
__global__ void k_wy_ts(int nbk, int nw, const z64 *T, const z64 *S, z64 *Sp) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nw * nbk) return;
    const int j = (int)(t / nbk), q = (int)(t - (int64_t)j * nbk);
    z64 acc = z64{0.0, 0.0};
    for (int r = q; r < nbk; ++r) acc = acc + cmul(T[q * nbk + r], S[(int64_t)j * nbk + r]);
    Sp[t] = acc;
}

// Diagonal block of the blocked Cholesky: factor G[j0 .. j0+jb)^2 in LDS (lower), write L11
// back and Li = L11^{-1} (jb x jb, row-major). Skipped when an earlier block failed.
__global__ __launch_bounds__(1024) void k_chol_diag(z64 *G, int ld, int j0, int jb, z64 *Li, int *info) {
    __shared__ z64 L[kCB][kCB + 1];
    __shared__ z64 X[kCB][kCB + 1];
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (j0 == 0 && tid == 0) *info = 0;
    if (tid == 0) bad = 0;
    __syncthreads();
    if (j0 > 0 && *info != 0) return;
    for (int t = tid; t < jb * jb; t += blockDim.x) {
        const int i = t / jb, j = t - i * jb;
        L[i][j] = j <= i ? G[(int64_t)(j0 + i) * ld + j0 + j] : z64{0.0, 0.0};
    }
    __syncthreads();
    for (int k = 0; k < jb; ++k) {
        const double dkk = L[k][k].re;
        if (!(dkk > 0.0) || !isfinite(dkk)) {
            if (tid == 0) {
                *info = j0 + k + 1;
                bad = 1;
            }
            __syncthreads();
            return;
        }
        const double lkk = sqrt(dkk), inv = 1.0 / lkk;
        __syncthreads();
        if (tid > k && tid < jb) L[tid][k] = z64{L[tid][k].re * inv, L[tid][k].im * inv};
        __syncthreads();
        if (tid == 0) L[k][k] = z64{lkk, 0.0};
        const int m = jb - k - 1;
        for (int t = tid; t < m * m; t += blockDim.x) {
            const int i = k + 1 + t / m, j = k + 1 + t % m;
            if (j <= i) L[i][j] = L[i][j] - cmulc(L[i][k], L[j][k]);
        }
        __syncthreads();
    }
    // Li = L^{-1} by forward substitution, one thread per column
    if (tid < jb) {
        const int c = tid;
        for (int i = 0; i < c; ++i) X[i][c] = z64{0.0, 0.0};
        X[c][c] = z64{1.0 / L[c][c].re, 0.0};
        for (int i = c + 1; i < jb; ++i) {
            z64 s = z64{0.0, 0.0};
            for (int q = c; q < i; ++q) s = s + cmul(L[i][q], X[q][c]);
            const double r = 1.0 / L[i][i].re;
            X[i][c] = z64{-s.re * r, -s.im * r};
        }
    }
    __syncthreads();
    for (int t = tid; t < jb * jb; t += blockDim.x) {
        const int i = t / jb, j = t - i * jb;
        if (j <= i) G[(int64_t)(j0 + i) * ld + j0 + j] = L[i][j];
        Li[t] = X[i][j];
    }
}

}  // namespace

// ------------------------------------------------------------------ drivers --

// Scratch of the large-order routines (bytes), carved in the order below.
size_t heev_large_scratch_bytes(int n, int nw) {
    const size_t zn = sizeof(z64);
    return 17 * 256                                       // alignment of the 17 regions
           + (size_t)n * (2 * sizeof(double) + zn)        // d, e, tau
           + (size_t)n * n * zn                           // Vr
           + (size_t)3 * n * 2 * kPL * zn                 // PX, PY, PXc
           + (size_t)2 * n * zn + 2 * kPL * zn            // vbuf, y, s
           + (size_t)n * n * sizeof(double)               // Z
           + (size_t)2 * kPL * kPL * zn                   // Gram, T
           + (size_t)2 * nw * kPL * zn                    // S, S'
           + std::max(gemm_cn_part_bytes(n, n, 2 * kPL, 16, 0), gemm_cn_part_bytes(kPL, nw, n, 16, 0))
           + 4096;
}

int stein_vectors(int n, const double *d, const double *e, int nw, const double *w, double *Z, int ldz, void *work,
                  size_t work_bytes, hipStream_t st);   // dense.hip
int stebz_values(int n, const double *d, const double *e, int nw, double *w, hipStream_t st);   // dense.hip
size_t stein_work_bytes(int n, int nw);   // dense.hip

int heev_lowest_large(int n, z64 *A, int ld, int nw, double *w, z64 *coef, int ldc, void *scratch,
                      hipStream_t st) {
    if (n > kMaxSub) return set_error(ABACUS_PW_EBAD_SHAPE, "subspace size above the device eigensolver limit");
    char *p = static_cast<char *>(scratch);
    auto take = [&](size_t bytes) {
        char *q = p;
        p += (bytes + 255) / 256 * 256;
        return q;
    };
    TrdArgs a;
    a.n = n;
    a.ld = ld;
    a.A = A;
    a.d = reinterpret_cast<double *>(take(sizeof(double) * n));
    a.e = reinterpret_cast<double *>(take(sizeof(double) * n));
    a.tau = reinterpret_cast<z64 *>(take(sizeof(z64) * n));
    a.Vr = reinterpret_cast<z64 *>(take(sizeof(z64) * (size_t)n * n));
    a.PX = reinterpret_cast<z64 *>(take(sizeof(z64) * (size_t)n * 2 * kPL));
    a.PY = reinterpret_cast<z64 *>(take(sizeof(z64) * (size_t)n * 2 * kPL));
    a.PXc = reinterpret_cast<z64 *>(take(sizeof(z64) * (size_t)n * 2 * kPL));
    a.vbuf = reinterpret_cast<z64 *>(take(sizeof(z64) * n));
    a.y = reinterpret_cast<z64 *>(take(sizeof(z64) * n));
    a.s = reinterpret_cast<z64 *>(take(sizeof(z64) * 2 * kPL));
    double *Z = reinterpret_cast<double *>(take(sizeof(double) * (size_t)n * n));
    z64 *Gt = reinterpret_cast<z64 *>(take(sizeof(z64) * kPL * kPL));
    z64 *T = reinterpret_cast<z64 *>(take(sizeof(z64) * kPL * kPL));
    z64 *S = reinterpret_cast<z64 *>(take(sizeof(z64) * (size_t)nw * kPL));
    z64 *Sp = reinterpret_cast<z64 *>(take(sizeof(z64) * (size_t)nw * kPL));
    void *part = take(std::max(gemm_cn_part_bytes(n, n, 2 * kPL, 16, 0), gemm_cn_part_bytes(kPL, nw, n, 16, 0)));
    {
        KernelTimer kt("hetrd_mc", st);
        for (int k0 = 0; k0 < n - 1; k0 += kPL) {
            const int bw = std::min(kPL, n - 1 - k0);
            if (bw < kPL) {
                // a partial panel: the columns it does not write must be zero for the trailing GEMM
                const int64_t cnt = (int64_t)n * 2 * kPL;
                hipLaunchKernelGGL(k_zero, dim3((unsigned)ceil_div64(cnt, 256)), dim3(256), 0, st, a.PX, cnt);
                hipLaunchKernelGGL(k_zero, dim3((unsigned)ceil_div64(cnt, 256)), dim3(256), 0, st, a.PY, cnt);
            }
            for (int c = 0; c < bw; ++c) {
                const int k = k0 + c, m = n - k - 1;
                hipLaunchKernelGGL(k_trd_col, dim3(1), dim3(kColThreads), 0, st, a, k0, c, 0);
                hipLaunchKernelGGL(k_trd_hemv, dim3((unsigned)ceil_div(m, 4)), dim3(256), sizeof(z64) * (size_t)m, st, a,
                                   k, c);
            }
            hipLaunchKernelGGL(k_trd_col, dim3(1), dim3(kColThreads), 0, st, a, k0, bw, 1);
            APW_TRY(check_launch("hetrd_mc panel"));
            const int t0 = k0 + bw, mt = n - t0;
            if (mt > 0)
                APW_TRY(gemm_cn(0, mt, mt, 2 * kPL, a.PY + (size_t)t0 * 2 * kPL, 2 * kPL, a.PX + (size_t)t0 * 2 * kPL,
                                2 * kPL, A + (size_t)t0 * ld + t0, ld, -1.0, 1.0, part, 0, st));
        }
        hipLaunchKernelGGL(k_trd_last, dim3(1), dim3(64), 0, st, A, ld, n, a.d);
        APW_TRY(check_launch("hetrd_mc last"));
    }
    APW_TRY(stebz_values(n, a.d, a.e, nw, w, st));
    {
        // inverse-iteration work space: its own region after the GEMM partials
        void *work = take(stein_work_bytes(n, nw));
        APW_TRY(stein_vectors(n, a.d, a.e, nw, w, Z, n, work, stein_work_bytes(n, nw), st));
    }
    KernelTimer kt("unmtr_mc", st);
    {
        const int64_t tot = (int64_t)n * nw;
        hipLaunchKernelGGL(k_real_rows, dim3((unsigned)ceil_div64(tot, 256)), dim3(256), 0, st, Z, n, n, nw, coef, ldc);
        APW_TRY(check_launch("real rows"));
    }
    // coef = H_0 ... H_{n-2} Z, blocks of kPL reflectors from the last block to the first
    const int nref = n - 1;
    for (int b0 = ((nref - 1) / kPL) * kPL; b0 >= 0; b0 -= kPL) {
        const int nbk = std::min(kPL, nref - b0);
        const z64 *Vb = a.Vr + (size_t)b0 * n;
        APW_TRY(gemm_cn(0, nbk, nbk, n, Vb, n, Vb, n, Gt, nbk, 1.0, 0.0, part, 0, st));
        hipLaunchKernelGGL(k_wy_t, dim3(1), dim3(kPL), 0, st, nbk, a.tau + b0, Gt, T);
        APW_TRY(gemm_cn(0, nbk, nw, n, Vb, n, coef, ldc, S, nbk, 1.0, 0.0, part, 0, st));
        const int64_t tot = (int64_t)nw * nbk;
        hipLaunchKernelGGL(k_wy_ts, dim3((unsigned)ceil_div64(tot, 256)), dim3(256), 0, st, nbk, nw, T, S, Sp);
        APW_TRY(check_launch("wy"));
        APW_TRY(gemm_nn(0, nw, n, nbk, Sp, nbk, Vb, n, coef, ldc, -1.0, 1.0, st));
    }
    return ABACUS_PW_OK;
}

size_t potrf_large_scratch_bytes(int n) {
    return (size_t)kCB * kCB * sizeof(z64) + (size_t)n * kCB * sizeof(z64) +
           gemm_cn_part_bytes(n, n, kCB, 16, 0) + gemm_cn_part_bytes(kCB, n, kCB, 16, 0) + 1024;
}

// Blocked Cholesky of G (lower triangle := L); *info_dev = 0 or (failed pivot + 1).
int potrf_large(int n, z64 *G, int ld, int *info_dev, void *scratch, hipStream_t st) {
    char *p = static_cast<char *>(scratch);
    z64 *Li = reinterpret_cast<z64 *>(p);
    z64 *tmp = Li + kCB * kCB;
    void *part = tmp + (size_t)n * kCB;
    KernelTimer kt("potrf_mc", st);
    for (int j0 = 0; j0 < n; j0 += kCB) {
        const int jb = std::min(kCB, n - j0), j1 = j0 + jb, m = n - j1;
        hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(1024), 0, st, G, ld, j0, jb, Li, info_dev);
        APW_TRY(check_launch("chol diag"));
        if (m == 0) break;
        // L21 = A21 L11^{-H}: tmp[i][q] = sum_r conj(Li[q][r]) A21[i][r]
        APW_TRY(gemm_cn(0, jb, m, jb, Li, jb, G + (size_t)j1 * ld + j0, ld, tmp, jb, 1.0, 0.0, part, 0, st));
        APW_HIP(hipMemcpy2DAsync(G + (size_t)j1 * ld + j0, sizeof(z64) * ld, tmp, sizeof(z64) * jb, sizeof(z64) * jb, m,
                                 hipMemcpyDeviceToDevice, st));
        // A22 -= L21 L21^H
        APW_TRY(gemm_cn(0, m, m, jb, G + (size_t)j1 * ld + j0, ld, G + (size_t)j1 * ld + j0, ld,
                        G + (size_t)j1 * ld + j1, ld, -1.0, 1.0, part, 0, st));
    }
    return ABACUS_PW_OK;
}

}  // namespace apw

// Small dense FP64 linear algebra on the GPU for the Davidson subspace
// (Sec. III.B names Davidson; its Rayleigh-Ritz and orthonormalisation steps
// need a Cholesky factorisation and a Hermitian eigensolver of the subspace
// matrix, kept in FP64 on the device):
//
//   k_potrf      Cholesky G = L L^H of a Hermitian positive definite matrix
//                (one work-group; k_potrf_lds keeps the packed triangle in LDS
//                for n <= 136).
//   k_trinv      the inverse L^{-1} (one wavefront per column).
//   k_hetrd      Householder reduction of a Hermitian matrix to a real
//                symmetric tridiagonal T = Q^H A Q (one work-group, blocked in
//                panels; the reflector convention H = I - tau v v^H, v[0] = 1,
//                makes every off-diagonal real).
//   k_stebz      eigenvalues of T by bisection on Sturm counts; one wavefront per
//                eigenvalue, each of its 64 lanes evaluating one point of a
//                65-way multisection of the current bracket.
//   k_stein      eigenvectors of T by inverse iteration (four solves from a
//                pseudo-random start) with a pivoted tridiagonal LU; eigenvalues
//                closer than 1e-7 ||T|| form a cluster handled by one thread,
//                which re-orthogonalises the cluster's vectors (modified
//                Gram-Schmidt) after every solve.
//                Between clusters inverse iteration leaves a non-orthogonality
//                of at most eps ||T|| / gap (2e-9); callers remove it with one
//                Lowdin step (see the Davidson driver).
//   k_unmtr      y = Q z for every wanted eigenvector (one wavefront each).
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
// Wave-wide sum (fixed butterfly order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// G (n x n, ld) Hermitian positive definite; its lower triangle is replaced
// by L with G = L L^H (right-looking, in global memory, one work-group).
// info = 0, or k + 1 when the k-th pivot is not positive.
__global__ __launch_bounds__(kNT) void k_potrf(int n, z64 *G, int ld, int *info) {
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
}

// The same factorisation with the packed lower triangle (row i at i (i+1) / 2)
// resident in LDS, for n <= kCholLds; L is written back to G at the end.
constexpr int kCholLds = 136;   // 136 * 137 / 2 complex128 = 148 KB of LDS
__host__ __device__ __forceinline__ int tri(int i) { return i * (i + 1) / 2; }

__global__ __launch_bounds__(kNT) void k_potrf_lds(int n, z64 *G, int ld, int *info) {
    extern __shared__ __align__(16) unsigned char smem[];
    z64 *Lp = reinterpret_cast<z64 *>(smem);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int i = wv; i < n; i += kNT / 64)
        for (int j = lane; j <= i; j += 64) Lp[tri(i) + j] = G[(int64_t)i * ld + j];
    __syncthreads();
    const int tx = tid & 31, ty = tid >> 5;
    for (int k = 0; k < n; ++k) {
        const double dkk = Lp[tri(k) + k].re;
        if (!(dkk > 0.0) || !isfinite(dkk)) {
            if (tid == 0) *info = k + 1;
            return;
        }
        const double lkk = sqrt(dkk), inv = 1.0 / lkk;
        for (int i = k + 1 + tid; i < n; i += kNT) {
            z64 &g = Lp[tri(i) + k];
            g = z64{g.re * inv, g.im * inv};
        }
        __syncthreads();
        if (tid == 0) Lp[tri(k) + k] = z64{lkk, 0.0};
        for (int i = k + 1 + ty; i < n; i += 32) {
            const z64 a = Lp[tri(i) + k];
            for (int j = k + 1 + tx; j <= i; j += 32) Lp[tri(i) + j] = Lp[tri(i) + j] - cmulc(a, Lp[tri(j) + k]);
        }
        __syncthreads();
    }
    for (int i = wv; i < n; i += kNT / 64)
        for (int j = lane; j <= i; j += 64) G[(int64_t)i * ld + j] = Lp[tri(i) + j];
    if (tid == 0) *info = 0;
}

// Linv = L^{-1} (lower triangular, zero above the diagonal) by forward
// substitution, one wavefront per column c: x_c = 1 / L_cc and
// x_i = -(sum_{c <= q < i} L_iq x_q) / L_ii, the sum over the contiguous row i
// of L split across the lanes (x_q in lane (q - c) % 64, slot (q - c) / 64),
// with row i + 1 loaded while row i is summed. Skipped when info != 0.
template <int R>
__global__ __launch_bounds__(256) void k_trinv(int n, const z64 *__restrict__ L, int ld, z64 *__restrict__ Linv,
                                               int ldi, const int *__restrict__ info) {
    if (*info != 0) return;
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= n) return;
    for (int i = lane; i < c; i += 64) Linv[(int64_t)i * ldi + c] = z64{0.0, 0.0};
    z64 x[R], cur[R], nxt[R];
#pragma unroll
    for (int t = 0; t < R; ++t) x[t] = z64{0.0, 0.0};
    const double xc = 1.0 / L[(int64_t)c * ld + c].re;
    if (lane == 0) {
        x[0] = z64{xc, 0.0};
        Linv[(int64_t)c * ldi + c] = x[0];
    }
    auto load_row = [&](int i, z64 *r) {
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int q = c + lane + 64 * t;
            r[t] = q < i ? L[(int64_t)i * ld + q] : z64{0.0, 0.0};
        }
    };
    double lnext = 1.0;
    if (c + 1 < n) {
        load_row(c + 1, nxt);
        lnext = L[(int64_t)(c + 1) * ld + c + 1].re;
    }
    for (int i = c + 1; i < n; ++i) {
        const double lii = lnext;
#pragma unroll
        for (int t = 0; t < R; ++t) cur[t] = nxt[t];
        if (i + 1 < n) {
            load_row(i + 1, nxt);
            lnext = L[(int64_t)(i + 1) * ld + i + 1].re;
        }
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const z64 p = cmul(cur[t], x[t]);
            sr += p.re;
            si += p.im;
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        const z64 xi = z64{-sr / lii, -si / lii};
        const int r = i - c;
#pragma unroll
        for (int t = 0; t < R; ++t)
            if ((r >> 6) == t && lane == (r & 63)) x[t] = xi;
        if (lane == 0) Linv[(int64_t)i * ldi + c] = xi;
    }
}

// ------------------------------------------------------------- tridiagonal --

constexpr int kPanel = 8;   // columns per panel of the blocked reduction
constexpr int kRows = 64;   // rows per LDS chunk of the trailing update
constexpr int kPanelLdsN = 256;   // largest n whose panel vectors V, W are kept in LDS
constexpr int kSymvBatch = 8;    // loads in flight per thread in the symmetric product

// A (n x n, ld) Hermitian, full storage. On exit d[n], e[n-1] hold T and
// column k of A below row k+1 holds v_k (v_k[k+1] = 1), tau[k] its factor,
// so Q = H_0 H_1 ... H_{n-2} with H_k = I - tau_k v_k v_k^H. Row k of Vr
// (n x n) receives the same v_k in columns k+1 .. n-1 (contiguous, for k_unmtr).
//
// Blocked as in LAPACK's panel reduction: inside a panel of kPanel columns the
// rank-2 updates A -= v w^H + w v^H are kept as the vectors V, W (VW scratch,
// 2 kPanel n) and applied to each column as it is reached; the symmetric
// product y = A22 v reads A22 as it was before the panel and subtracts
// V (W^H v) + W (V^H v); the trailing matrix takes all the panel's updates in
// one pass. Since v = [1, scale * x] is linear in the reflector's scale, the
// product and the dot products with V and W start from the raw column x in the
// same pass as its norm, leaving four barriers per column.
template <bool kLdsPanel>
__global__ __launch_bounds__(kNT) void k_hetrd(int n, z64 *A, int ld, double *d, double *e, z64 *tau, z64 *VW,
                                               z64 *Vr) {
    __shared__ z64 xs[kSmallSub];      // column k from the diagonal down, panel updates applied
    __shared__ z64 a0s[kSmallSub];     // first column of A22 (conjugated row)
    __shared__ z64 part[kNT];          // partial sums of A22 x
    __shared__ z64 dots[2 * kPanel];   // W^H x, V^H x over rows k+2 ..
    __shared__ z64 ybc;                // y_0, for the next column's update
    __shared__ double red[kNT / 64], red2[2][kNT / 64];
    __shared__ z64 rowvw[2 * kPanel][kRows];   // V then W, rows r0 .. r0 + kRows of the trailing update
    __shared__ z64 vw_lds[kLdsPanel ? 2 * kPanel * kPanelLdsN : 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = kNT / 64;
    // column q of the panel at [q * n + row]; in LDS (n <= kPanelLdsN) or in VW
    z64 *Vp = kLdsPanel ? vw_lds : VW;
    z64 *Wp = Vp + (int64_t)kPanel * n;
    for (int k0 = 0; k0 < n - 1; k0 += kPanel) {
        const int bw = min(kPanel, n - 1 - k0);
        for (int c = 0; c < bw; ++c) {
            const int k = k0 + c, m = n - k - 1;
            // P1 (first column of a panel): column k, rows k .. n-1, as stored.
            // Later columns of the panel are formed at the end of the previous one.
            if (c == 0) {
                if (tid <= m) xs[tid] = A[(int64_t)(k + tid) * ld + k];
                __syncthreads();
            }
            // P2: |x|^2, V^H x, W^H x and A22 x over x = xs[2 .. m] (v without its leading 1)
            const int mp = (m + 63) / 64 * 64, G = kNT / mp;
            z64 *A22 = A + (int64_t)(k + 1) * ld + k + 1;
            {
                double p = 0.0;
                for (int r = 2 + tid; r <= m; r += kNT) p += zabs2(xs[r]);
                p = wave_sum(p);
                if (lane == 0) red[wv] = p;
                for (int q = wv; q < 2 * c; q += nwv) {
                    const z64 *col = (q < c ? Wp + q * n : Vp + (q - c) * n) + k + 1;
                    double sr = 0.0, si = 0.0;
                    for (int j0 = 1 + lane; j0 < m; j0 += 4 * 64) {
                        z64 cv[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) cv[u] = j0 + 64 * u < m ? col[j0 + 64 * u] : z64{0.0, 0.0};
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            if (j0 + 64 * u < m) {
                                const z64 t = cmulc(xs[1 + j0 + 64 * u], cv[u]);   // conj(col) x
                                sr += t.re;
                                si += t.im;
                            }
                    }
                    sr = wave_sum(sr);
                    si = wave_sum(si);
                    if (lane == 0) dots[q] = z64{sr, si};
                }
                const int i = tid % mp, g = tid / mp;
                z64 acc = z64{0.0, 0.0};
                if (g < G && i < m) {
                    for (int j0 = 1 + g; j0 < m; j0 += kSymvBatch * G) {
                        z64 av[kSymvBatch];
#pragma unroll
                        for (int u = 0; u < kSymvBatch; ++u) {
                            const int j = min(j0 + u * G, m - 1);   // clamped: loads issue unconditionally
                            av[u] = A22[(int64_t)j * ld + i];
                        }
#pragma unroll
                        for (int u = 0; u < kSymvBatch; ++u) {
                            const int j = j0 + u * G;
                            if (j < m) acc = acc + cmul(zconj(av[u]), xs[1 + j]);
                        }
                    }
                    if (g == 0) a0s[i] = zconj(A22[i]);
                }
                part[tid] = acc;
            }
            __syncthreads();
            // P3: reflector, y = tau (A22 v - V (W^H v) - W (V^H v))
            double xn2 = 0.0;
            for (int q = 0; q < nwv; ++q) xn2 += red[q];
            const z64 alpha = xs[1];
            double beta = alpha.re;
            z64 t = z64{0.0, 0.0}, scale = z64{0.0, 0.0};
            if (!(xn2 == 0.0 && alpha.im == 0.0)) {
                beta = -copysign(sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn2), alpha.re);
                t = z64{(beta - alpha.re) / beta, -alpha.im / beta};
                const z64 den = z64{alpha.re - beta, alpha.im};   // scale = 1 / (alpha - beta)
                const double dd = zabs2(den);
                scale = z64{den.re / dd, -den.im / dd};
            }
            z64 vi = z64{0.0, 0.0}, yi = z64{0.0, 0.0};
            double pr = 0.0, pi = 0.0;
            if (tid < m) {
                const int i = tid;
                vi = i == 0 ? z64{1.0, 0.0} : cmul(xs[1 + i], scale);
                z64 s = z64{0.0, 0.0};
                for (int g = 0; g < G; ++g) s = s + part[g * mp + i];
                z64 y = a0s[i] + cmul(scale, s);
                for (int q = 0; q < c; ++q) {
                    const z64 wv_ = zconj(Wp[q * n + k + 1]) + cmul(scale, dots[q]);       // W^H v
                    const z64 vv_ = zconj(Vp[q * n + k + 1]) + cmul(scale, dots[c + q]);   // V^H v
                    y = y - cmul(Vp[q * n + k + 1 + i], wv_) - cmul(Wp[q * n + k + 1 + i], vv_);
                }
                yi = cmul(t, y);
                if (i == 0) ybc = yi;
                const z64 cv = cmulc(vi, yi);   // conj(y) v
                pr = cv.re;
                pi = cv.im;
            }
            pr = wave_sum(pr);
            pi = wave_sum(pi);
            if (lane == 0) {
                red2[0][wv] = pr;
                red2[1][wv] = pi;
            }
            __syncthreads();
            // P4: w = y - 1/2 tau (y^H v) v; store v, w and the reflector. Inside a
            // panel, thread i also forms row k+1+i of the next column: as stored
            // it is A22[i][0] = a0s[i] (A22 is Hermitian and untouched by this
            // panel), minus the updates of panel columns 0 .. c, whose entries in
            // row k+1 are W[c][k+1] = w_0 = y_0 + a2 and V[c][k+1] = 1.
            double sr = 0.0, si = 0.0;
            for (int q = 0; q < nwv; ++q) {
                sr += red2[0][q];
                si += red2[1][q];
            }
            const z64 a2 = cmul(z64{-0.5 * t.re, -0.5 * t.im}, z64{sr, si});
            if (tid == 0) {
                d[k] = xs[0].re;
                e[k] = beta;
                tau[k] = t;
            }
            if (tid < m) {
                const int i = tid;
                const z64 wi = yi + cmul(a2, vi);
                Wp[c * n + k + 1 + i] = wi;
                Vp[c * n + k + 1 + i] = vi;
                A[(int64_t)(k + 1 + i) * ld + k] = vi;
                Vr[(int64_t)k * n + k + 1 + i] = vi;
                if (c + 1 < bw) {
                    const z64 w0 = ybc + a2;
                    z64 a = a0s[i] - cmulc(vi, w0) - wi;   // q = c: v_i conj(w_0) + w_i conj(1)
                    for (int q = 0; q < c; ++q)
                        a = a - cmulc(Vp[q * n + k + 1 + i], Wp[q * n + k + 1]) -
                            cmulc(Wp[q * n + k + 1 + i], Vp[q * n + k + 1]);
                    xs[i] = a;
                }
            }
            __syncthreads();
        }
        // trailing matrix A[t0:, t0:] -= V W^H + W V^H over the panel: a thread
        // keeps its column's panel values in registers; the rows' values pass
        // through LDS in chunks of kRows
        const int t0 = k0 + bw, mt = n - t0;
        const int mtp = (mt + 63) / 64 * 64, G = kNT / mtp;
        const int jj = tid % mtp, g = tid / mtp;
        const bool mine = g < G && jj < mt;
        z64 vj[kPanel], wj[kPanel];
#pragma unroll
        for (int q = 0; q < kPanel; ++q) {
            vj[q] = mine && q < bw ? zconj(Vp[q * n + t0 + jj]) : z64{0.0, 0.0};
            wj[q] = mine && q < bw ? zconj(Wp[q * n + t0 + jj]) : z64{0.0, 0.0};
        }
        for (int r0 = t0; r0 < n; r0 += kRows) {
            const int nr = min(kRows, n - r0);
            for (int idx = tid; idx < 2 * kPanel * kRows; idx += kNT) {
                const int q2 = idx / kRows, r = idx - q2 * kRows, q = q2 % kPanel;
                const z64 *src = q2 < kPanel ? Vp + q * n : Wp + q * n;
                rowvw[q2][r] = q < bw && r < nr ? src[r0 + r] : z64{0.0, 0.0};
            }
            __syncthreads();
            if (mine)
                for (int rb = g; rb < nr; rb += 2 * G) {
                    z64 a[2];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int r = rb + u * G;
                        a[u] = r < nr ? A[(int64_t)(r0 + r) * ld + t0 + jj] : z64{0.0, 0.0};
                    }
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int r = rb + u * G;
                        if (r < nr) {
                            z64 s0 = z64{0.0, 0.0}, s1 = z64{0.0, 0.0};   // two independent chains
#pragma unroll
                            for (int q = 0; q < kPanel; ++q) {
                                s0 = s0 + cmul(rowvw[q][r], wj[q]);
                                s1 = s1 + cmul(rowvw[kPanel + q][r], vj[q]);
                            }
                            A[(int64_t)(r0 + r) * ld + t0 + jj] = a[u] - (s0 + s1);
                        }
                    }
                }
            __syncthreads();
        }
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
// One thread per eigenvalue (the first of each cluster handles its cluster).
// The serial recurrences of the factorisation and the two triangular solves
// carry their running values in registers; only their outputs go to memory,
// so no step waits on a load of what the previous step stored. The per-thread
// work arrays are interleaved (element i of thread j at i * S + j, S threads)
// so that a wavefront's accesses at one i are contiguous.
// scratch: 6 n S doubles, S = gridDim.x * blockDim.x.
constexpr int kCh = 8;   // steps per prefetched chunk of the inverse-iteration recurrences

__global__ __launch_bounds__(64) void k_stein(int n, const double *__restrict__ d, const double *__restrict__ e, int nw,
                                              const double *__restrict__ w, double *__restrict__ Z, int ldz,
                                              double *__restrict__ scratch) {
    __shared__ double ds[kMaxSub], es[kMaxSub];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        ds[i] = d[i];
        es[i] = i < n - 1 ? e[i] : 0.0;
    }
    __syncthreads();
    const int S = gridDim.x * blockDim.x;
    const int j0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (j0 >= nw) return;
    double anorm = 0.0;
    for (int i = 0; i < n; ++i)
        anorm = fmax(anorm, fabs(ds[i]) + (i > 0 ? fabs(es[i - 1]) : 0.0) + (i < n - 1 ? fabs(es[i]) : 0.0));
    const double eps = 2.220446049250313e-16;
    const double ortol = kClusterTol * anorm;
    if (j0 > 0 && w[j0] - w[j0 - 1] <= ortol) return;   // not the first of its cluster
    int j1 = j0 + 1;
    while (j1 < nw && w[j1] - w[j1 - 1] <= ortol) ++j1;
    // U = [rd (1/pivot), du, du2], L = [dl], row interchanges piv; x the iterate
    double *rd = scratch + j0, *dl = rd + (int64_t)n * S, *du = dl + (int64_t)n * S, *du2 = du + (int64_t)n * S;
    double *piv = du2 + (int64_t)n * S, *x = piv + (int64_t)n * S;
    const double tiny = eps * fmax(anorm, 1e-300);
    auto guard = [tiny](double v) { return fabs(v) < tiny ? copysign(tiny, v == 0.0 ? 1.0 : v) : v; };
    double lam_prev = 0.0;
    for (int j = j0; j < j1; ++j) {
        double lam = w[j];
        const double sep = 10.0 * eps * fmax(fabs(lam), anorm * eps);
        if (j > j0 && lam - lam_prev < sep) lam = lam_prev + sep;
        lam_prev = lam;
        // LU of T - lam I with partial pivoting (rows i and i+1 swap when |sub| > |diag|)
        double cd = ds[0] - lam, cu = n > 1 ? es[0] : 0.0;
        for (int i = 0; i < n - 1; ++i) {
            const double sub = es[i], dn = ds[i + 1] - lam, un = i < n - 2 ? es[i + 1] : 0.0;
            const int64_t o = (int64_t)i * S;
            if (fabs(cd) >= fabs(sub)) {
                const double p = guard(cd), f = sub / p;
                rd[o] = 1.0 / p;
                dl[o] = f;
                du[o] = cu;
                du2[o] = 0.0;
                piv[o] = 0.0;
                cd = dn - f * cu;
                cu = un;
            } else {
                const double f = cd / sub;
                rd[o] = 1.0 / sub;
                dl[o] = f;
                du[o] = dn;
                du2[o] = un;
                piv[o] = 1.0;
                cd = cu - f * dn;
                cu = -f * un;
            }
        }
        rd[(int64_t)(n - 1) * S] = 1.0 / guard(cd);
        // inverse iteration from a pseudo-random start; the iterate is renormalised
        // lazily (the solve is linear, so the scale sc is applied as it is read).
        // Loads run a chunk of kCh steps ahead of the recurrences.
        double sc = 1.0;
        for (int it = 0; it < 4; ++it) {
            // forward: L y = P b. Loads are unconditional (indices clamped into
            // the arrays) so that a chunk's loads are all in flight together.
            double cur = it == 0 ? hash_uniform((unsigned)j, 0u) : sc * x[0];
            if (n > 1) {
                double fa[kCh], fp[kCh], fb[kCh], na[kCh], np[kCh], nb_[kCh];
                auto fetch = [&](int i0, double *a, double *pv, double *b) {
#pragma unroll
                    for (int u = 0; u < kCh; ++u) {
                        const int64_t o = (int64_t)min(i0 + u, n - 2) * S;
                        a[u] = dl[o];
                        pv[u] = piv[o];
                        b[u] = x[o + S];
                    }
                };
                fetch(0, na, np, nb_);
                for (int i0 = 0; i0 < n - 1; i0 += kCh) {
#pragma unroll
                    for (int u = 0; u < kCh; ++u) {
                        fa[u] = na[u];
                        fp[u] = np[u];
                        fb[u] = nb_[u];
                    }
                    if (i0 + kCh < n - 1) fetch(i0 + kCh, na, np, nb_);
#pragma unroll
                    for (int u = 0; u < kCh; ++u) {
                        const int i = i0 + u;
                        if (i < n - 1) {
                            const double b = it == 0 ? hash_uniform((unsigned)j, (unsigned)(i + 1)) : sc * fb[u];
                            const bool sw = fp[u] != 0.0;
                            x[(int64_t)i * S] = sw ? b : cur;
                            cur = sw ? cur - fa[u] * b : b - fa[u] * cur;
                        }
                    }
                }
            }
            // backward: U x = y
            double x1 = cur * rd[(int64_t)(n - 1) * S], x2 = 0.0;
            x[(int64_t)(n - 1) * S] = x1;
            double amax = fabs(x1);
            if (n > 1) {
                double bx[kCh], bu[kCh], bu2[kCh], br[kCh], nx[kCh], nu[kCh], nu2[kCh], nr[kCh];
                auto fetch = [&](int i0, double *xx, double *u1, double *u2, double *r) {
#pragma unroll
                    for (int u = 0; u < kCh; ++u) {
                        const int64_t o = (int64_t)max(i0 - u, 0) * S;
                        xx[u] = x[o];
                        u1[u] = du[o];
                        u2[u] = du2[o];
                        r[u] = rd[o];
                    }
                };
                fetch(n - 2, nx, nu, nu2, nr);
                for (int i0 = n - 2; i0 >= 0; i0 -= kCh) {
#pragma unroll
                    for (int u = 0; u < kCh; ++u) {
                        bx[u] = nx[u];
                        bu[u] = nu[u];
                        bu2[u] = nu2[u];
                        br[u] = nr[u];
                    }
                    if (i0 - kCh >= 0) fetch(i0 - kCh, nx, nu, nu2, nr);
#pragma unroll
                    for (int u = 0; u < kCh; ++u) {
                        const int i = i0 - u;
                        if (i >= 0) {
                            const double xi = (bx[u] - bu[u] * x1 - bu2[u] * x2) * br[u];
                            x[(int64_t)i * S] = xi;
                            amax = fmax(amax, fabs(xi));
                            x2 = x1;
                            x1 = xi;
                        }
                    }
                }
            }
            // re-orthogonalise inside the cluster
            for (int q = j0; q < j; ++q) {
                double s = 0.0;
                for (int i = 0; i < n; ++i) s += Z[(int64_t)q * ldz + i] * x[(int64_t)i * S];
                for (int i = 0; i < n; ++i) x[(int64_t)i * S] -= s * Z[(int64_t)q * ldz + i];
                amax = 0.0;
                for (int i = 0; i < n; ++i) amax = fmax(amax, fabs(x[(int64_t)i * S]));
            }
            double s2 = 0.0;
            const double ra = 1.0 / amax;
            for (int i0 = 0; i0 < n; i0 += kCh) {
                double t[kCh];
#pragma unroll
                for (int u = 0; u < kCh; ++u) t[u] = x[(int64_t)min(i0 + u, n - 1) * S];
#pragma unroll
                for (int u = 0; u < kCh; ++u) t[u] = i0 + u < n ? t[u] * ra : 0.0;
#pragma unroll
                for (int u = 0; u < kCh; ++u) s2 += t[u] * t[u];
            }
            sc = ra / sqrt(s2);
        }
        for (int i = 0; i < n; ++i) Z[(int64_t)j * ldz + i] = sc * x[(int64_t)i * S];
    }
}

// coef[j*ldc + i] = (Q z_j)[i]: apply H_{n-2} .. H_0 to each real eigenvector.
// One wavefront per eigenvector, its entries i = lane + 64 t held in registers
// (R = ceil(n / 64) per lane); the next reflector's row of Vr is loaded while
// the current one is applied.
template <int R>
__global__ __launch_bounds__(256) void k_unmtr(int n, const z64 *__restrict__ Vr, const z64 *__restrict__ tau,
                                               const double *__restrict__ Z, int ldz, int nw, z64 *__restrict__ coef,
                                               int ldc) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= nw) return;
    z64 y[R], vc[R], vn[R];
    auto load_v = [&](int k, z64 *v) {
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int i = lane + 64 * t;
            v[t] = i > k + 1 && i < n ? Vr[(int64_t)k * n + i] : z64{i == k + 1 ? 1.0 : 0.0, 0.0};
        }
    };
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int i = lane + 64 * t;
        y[t] = z64{i < n ? Z[(int64_t)j * ldz + i] : 0.0, 0.0};
    }
    if (n >= 2) load_v(n - 2, vn);
    for (int k = n - 2; k >= 0; --k) {
#pragma unroll
        for (int t = 0; t < R; ++t) vc[t] = vn[t];
        if (k > 0) load_v(k - 1, vn);
        const z64 tk = tau[k];
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const z64 c = cmulc(y[t], vc[t]);   // conj(v) y
            sr += c.re;
            si += c.im;
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        const z64 ts = cmul(tk, z64{sr, si});
#pragma unroll
        for (int t = 0; t < R; ++t) y[t] = y[t] - cmul(vc[t], ts);
    }
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int i = lane + 64 * t;
        if (i < n) coef[(int64_t)j * ldc + i] = y[t];
    }
}

// ---------------------------------------------------------------- drivers --
size_t potrf_large_scratch_bytes(int n);                                       // dense_large.hip
int potrf_large(int n, z64 *G, int ld, int *info_dev, void *scratch, hipStream_t st);
size_t heev_large_scratch_bytes(int n, int nw);
int heev_lowest_large(int n, z64 *A, int ld, int nw, double *w, z64 *coef, int ldc, void *scratch, hipStream_t st);

size_t potrf_scratch_bytes(int n) { return n >= kLargeCholMin ? potrf_large_scratch_bytes(n) : 256; }

int potrf_inv(int n, z64 *G, int ld, z64 *Linv, int ldi, int *info_dev, void *scratch, hipStream_t st) {
    if (n > kMaxChol) return set_error(ABACUS_PW_EBAD_SHAPE, "Cholesky size above the device limit (1024)");
    if (n >= kLargeCholMin) {
        APW_TRY(potrf_large(n, G, ld, info_dev, scratch, st));
    } else {
        KernelTimer kt("potrf_inv", st);
        if (n <= kCholLds) {
            const size_t lds = sizeof(z64) * (size_t)tri(n);
            static bool attr = false;
            if (!attr) {
                APW_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(k_potrf_lds),
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)(sizeof(z64) * (size_t)tri(kCholLds))));
                attr = true;
            }
            hipLaunchKernelGGL(k_potrf_lds, dim3(1), dim3(kNT), lds, st, n, G, ld, info_dev);
        } else {
            hipLaunchKernelGGL(k_potrf, dim3(1), dim3(kNT), 0, st, n, G, ld, info_dev);
        }
        APW_TRY(check_launch("potrf"));
    }
    KernelTimer kt("trinv", st);
    const dim3 grid(ceil_div(n, 4)), block(256);
    const int R = ceil_div(n, 64);
    if (R <= 1) hipLaunchKernelGGL(k_trinv<1>, grid, block, 0, st, n, G, ld, Linv, ldi, info_dev);
    else if (R <= 2) hipLaunchKernelGGL(k_trinv<2>, grid, block, 0, st, n, G, ld, Linv, ldi, info_dev);
    else if (R <= 4) hipLaunchKernelGGL(k_trinv<4>, grid, block, 0, st, n, G, ld, Linv, ldi, info_dev);
    else if (R <= 8) hipLaunchKernelGGL(k_trinv<8>, grid, block, 0, st, n, G, ld, Linv, ldi, info_dev);
    else hipLaunchKernelGGL(k_trinv<16>, grid, block, 0, st, n, G, ld, Linv, ldi, info_dev);
    return check_launch("trinv");
}

static int stein_slots(int nw) { return ceil_div(nw, 64) * 64; }

size_t stein_work_bytes(int n, int nw) { return (size_t)6 * n * stein_slots(nw) * sizeof(double) + 256; }

int stebz_values(int n, const double *d, const double *e, int nw, double *w, hipStream_t st) {
    KernelTimer kt("stebz", st);
    hipLaunchKernelGGL(k_stebz, dim3(ceil_div(nw, 4)), dim3(256), 0, st, n, d, e, nw, w);
    return check_launch("stebz");
}

int stein_vectors(int n, const double *d, const double *e, int nw, const double *w, double *Z, int ldz, void *work,
                  size_t work_bytes, hipStream_t st) {
    if (work_bytes < stein_work_bytes(n, nw)) return set_error(ABACUS_PW_EINTERNAL, "inverse-iteration work space");
    KernelTimer kt("stein", st);
    hipLaunchKernelGGL(k_stein, dim3(ceil_div(nw, 64)), dim3(64), 0, st, n, d, e, nw, w, Z, ldz,
                       static_cast<double *>(work));
    return check_launch("stein");
}

// Small orders: d, e (n doubles each), tau (n), the panel vectors V, W of the tridiagonal
// reduction (2 kPanel n), the reflector rows Vr (n x n), Z (n x n doubles) and the
// inverse-iteration arrays (6 n S doubles). Large orders: the layout of dense_large.hip.
size_t heev_scratch_bytes(int n) {
    if (n >= kLargeHeevMin) return heev_large_scratch_bytes(n, n) + stein_work_bytes(n, n) + 256;
    return (size_t)n * (2 * sizeof(double) + sizeof(z64)) + (size_t)2 * kPanel * n * sizeof(z64) +
           (size_t)n * n * sizeof(z64) + (size_t)n * n * sizeof(double) + stein_work_bytes(n, n) + 1024;
}

int heev_lowest(int n, z64 *A, int ld, int nw, double *w, z64 *coef, int ldc, void *scratch, hipStream_t st) {
    if (n > kMaxSub) return set_error(ABACUS_PW_EBAD_SHAPE, "subspace size above the device eigensolver limit (4096)");
    if (n >= kLargeHeevMin) return heev_lowest_large(n, A, ld, nw, w, coef, ldc, scratch, st);
    char *s = static_cast<char *>(scratch);
    double *d = reinterpret_cast<double *>(s);
    double *e = d + n;
    z64 *tau = reinterpret_cast<z64 *>(e + n);
    z64 *VW = tau + n;
    z64 *Vr = VW + (size_t)2 * kPanel * n;
    double *Z = reinterpret_cast<double *>(Vr + (size_t)n * n);
    double *work = Z + (size_t)n * n;
    {
        KernelTimer kt("hetrd", st);
        if (n <= kPanelLdsN) hipLaunchKernelGGL(k_hetrd<true>, dim3(1), dim3(kNT), 0, st, n, A, ld, d, e, tau, VW, Vr);
        else hipLaunchKernelGGL(k_hetrd<false>, dim3(1), dim3(kNT), 0, st, n, A, ld, d, e, tau, VW, Vr);
        APW_TRY(check_launch("hetrd"));
    }
    APW_TRY(stebz_values(n, d, e, nw, w, st));
    APW_TRY(stein_vectors(n, d, e, nw, w, Z, n, work, stein_work_bytes(n, nw), st));
    {
        KernelTimer kt("unmtr", st);
        const dim3 grid(ceil_div(nw, 4)), block(256);
        const int R = ceil_div(n, 64);
        if (R <= 1) hipLaunchKernelGGL(k_unmtr<1>, grid, block, 0, st, n, Vr, tau, Z, n, nw, coef, ldc);
        else if (R <= 2) hipLaunchKernelGGL(k_unmtr<2>, grid, block, 0, st, n, Vr, tau, Z, n, nw, coef, ldc);
        else if (R <= 4) hipLaunchKernelGGL(k_unmtr<4>, grid, block, 0, st, n, Vr, tau, Z, n, nw, coef, ldc);
        else if (R <= 8) hipLaunchKernelGGL(k_unmtr<8>, grid, block, 0, st, n, Vr, tau, Z, n, nw, coef, ldc);
        else hipLaunchKernelGGL(k_unmtr<16>, grid, block, 0, st, n, Vr, tau, Z, n, nw, coef, ldc);
        APW_TRY(check_launch("unmtr"));
    }
    return ABACUS_PW_OK;
}

}  // namespace apw

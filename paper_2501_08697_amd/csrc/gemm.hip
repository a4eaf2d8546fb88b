// Complex GEMMs on the matrix cores (MFMA) for the Kleinman-Bylander term
// sum_ij |beta_i> D_ij <beta_j| psi (Sec. II.A) and for the Davidson subspace
// products. Two shapes cover every use, both with K-contiguous row vectors:
//
//   CN  C[j][i] = alpha * sum_k conj(A[i][k]) B[j][k] + beta * C[j][i]
//       (projections <a_i|b_j>; K = npw is long, so K is split across
//        work-groups and the partial tiles are summed in a fixed order)
//   NN  C[j][g] = alpha * sum_i A[j][i] B[i][g] + beta * C[j][g]
//       (combinations of basis vectors: Y += B Q, Psi = V Y)
//
// Tiles: a 256-thread work-group owns a 64 x 64 output tile; each of its four
// waves a 32 x 32 quarter as 2 x 2 blocks of 16 x 16 MFMA results. A complex
// product takes three real products (3M: ar br, ai bi and the product of the
// sums, from which the real and imaginary parts follow), so each block keeps
// three accumulators. Operands are staged in LDS (16 k per stage). FP64 uses v_mfma_f64_16x16x4f64, FP32 v_mfma_f32_16x16x4f32;
// both take one value of A and of B per lane (A[i][k] at lane i + 16 k, B[k][j]
// at lane j + 16 k) and return four values per lane in column j = lane % 16.
// The row of element e differs: the FP64 instruction interleaves rows
// (i = lane / 16 + 4 e), the FP32 one blocks them (i = 4 (lane / 16) + e);
// Acc<T>::row encodes this (measured on gfx950).
#include <algorithm>

#include "common.hpp"
#include "gemm.hpp"

namespace apw {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
template <> struct Acc<double> {
    using V = d4;
    __device__ static V zero() { return V{0.0, 0.0, 0.0, 0.0}; }
    __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int e) { return (lane >> 4) + 4 * e; }
};
template <> struct Acc<float> {
    using V = f4;
    __device__ static V zero() { return V{0.f, 0.f, 0.f, 0.f}; }
    __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int e) { return 4 * (lane >> 4) + e; }
};

constexpr int TM = 64, TN = 64, KT = 16, KP = KT + 1;
// Asking for at least two waves per SIMD makes the compiler keep the twelve
// accumulator blocks in ordinary VGPRs (166 in FP64, three waves per SIMD)
// instead of spreading them over VGPRs and AGPRs (278, one wave per SIMD).
constexpr int kGemmWaves = 2;

// ----------------------------------------------------------------- CN ------
// part[s][j][i] = sum over k in split s of conj(A[i][k]) B[j][k]
// TS is the type operands are stored in; they are rounded to T while staged
// (FP32 products of FP64 vectors for the reduced-precision subspace projection).
// Tile order: the blocks of one K chunk are logically consecutive (and so share an XCD's
// L2); inside a chunk they run in groups of gm row tiles by every column tile, so the
// tiles that run at the same time read few distinct A and B tiles while they move
// through K together (with the row tiles fastest, a chunk of a 2304 x 1024 product
// kept all 36 A tiles in flight and read 15.7x the operands).
template <typename T, typename TS = T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kGemmWaves))) void k_gemm_cn_part(int M, int N, int K, int kchunk, const cx<TS> *__restrict__ A,
                                                      int64_t lda, const cx<TS> *__restrict__ B, int64_t ldb,
                                                      cx<T> *__restrict__ part, int gm) {
    __shared__ cx<T> As[TM][KP];
    __shared__ cx<T> Bs[TN][KP];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int bx, by, bz;
    xcd_block(bx, by, bz);   // the tiles of one K chunk share an L2
    const int nm = gridDim.x, nn = gridDim.y;
    const int t = bx + nm * by;                        // tile of the chunk, in logical order
    const int grp = t / (gm * nn), first = grp * gm, rows = min(gm, nm - first);
    const int r = t - grp * gm * nn;
    const int i0 = (first + r % rows) * TM, j0 = (r / rows) * TN, s = bz;
    const int kb = s * kchunk, ke = min(K, kb + kchunk);
    using AV = typename Acc<T>::V;
    AV c1[2][2], c2[2][2], c3[2][2];   // sums of ar br, ai bi, (ar - ai)(br + bi)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) c1[a][b] = c2[a][b] = c3[a][b] = Acc<T>::zero();
    const int lr = tid >> 2, lk = (tid & 3) * 4;   // loader: row, first k of 4
    const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
    // loader rows past M (N) read the last row instead: they only feed outputs that are
    // never stored, and a whole stage then loads with no per-load branch (only the k tail
    // of a chunk is bounded, and zero-filled, since it enters every sum)
    const cx<TS> *ga = A + (int64_t)min(i0 + lr, M - 1) * lda + lk;
    const cx<TS> *gb = B + (int64_t)min(j0 + lr, N - 1) * ldb + lk;
    cx<T> ra[4], rb[4];
    auto load = [&](int k0) {
        if (k0 + KT <= ke) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ra[q] = cvt<T>(ga[k0 + q]);
                rb[q] = cvt<T>(gb[k0 + q]);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool in = k0 + lk + q < ke;
                ra[q] = in ? cvt<T>(ga[k0 + q]) : cx<T>{T(0), T(0)};
                rb[q] = in ? cvt<T>(gb[k0 + q]) : cx<T>{T(0), T(0)};
            }
        }
    };
    load(kb);
    for (int k0 = kb; k0 < ke; k0 += KT) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[lr][lk + q] = ra[q];
            Bs[lr][lk + q] = rb[q];
        }
        __syncthreads();
        if (k0 + KT < ke) load(k0 + KT);   // next stage in flight while this one multiplies
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kk = 4 * q + (lane >> 4);
            cx<T> a[2], b[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) a[r] = As[wi + 16 * r + (lane & 15)][kk];
#pragma unroll
            for (int c = 0; c < 2; ++c) b[c] = Bs[wj + 16 * c + (lane & 15)][kk];
            T as[2], bs[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) as[r] = a[r].re - a[r].im;
#pragma unroll
            for (int c = 0; c < 2; ++c) bs[c] = b[c].re + b[c].im;
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    // conj(a) b with three real products:
                    //   re = ar br + ai bi,  im = (ar - ai)(br + bi) - ar br + ai bi
                    c1[r][c] = Acc<T>::mma(a[r].re, b[c].re, c1[r][c]);
                    c2[r][c] = Acc<T>::mma(a[r].im, b[c].im, c2[r][c]);
                    c3[r][c] = Acc<T>::mma(as[r], bs[c], c3[r][c]);
                }
        }
        __syncthreads();
    }
    cx<T> *out = part + (int64_t)s * N * M;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int gj = j0 + wj + 16 * c + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gi = i0 + wi + 16 * r + Acc<T>::row(lane, e);
                if (gi < M && gj < N)
                    out[(int64_t)gj * M + gi] = cx<T>{c1[r][c][e] + c2[r][c][e], c3[r][c][e] - c1[r][c][e] + c2[r][c][e]};
            }
        }
}

// C[j][i] = alpha * sum_s part[s][j][i] + beta * C[j][i]   (fixed summation order)
template <typename T, typename TC = T>
__global__ void k_reduce(int M, int N, int nsplit, const cx<T> *__restrict__ part, cx<TC> *__restrict__ C, int64_t ldc,
                         double alpha, double beta) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)M * N) return;
    const int j = (int)(idx / M), i = (int)(idx - (int64_t)j * M);
    const int64_t ss = (int64_t)M * N;
    double r4[4] = {0.0, 0.0, 0.0, 0.0}, i4[4] = {0.0, 0.0, 0.0, 0.0};   // four independent chains
    int s = 0;
    for (; s + 3 < nsplit; s += 4) {
        cx<T> v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = part[(int64_t)(s + u) * ss + idx];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            r4[u] += (double)v[u].re;
            i4[u] += (double)v[u].im;
        }
    }
    for (int u = 0; s < nsplit; ++s, ++u) {
        const cx<T> v = part[(int64_t)s * ss + idx];
        r4[u] += (double)v.re;
        i4[u] += (double)v.im;
    }
    double re = (r4[0] + r4[1]) + (r4[2] + r4[3]), im = (i4[0] + i4[1]) + (i4[2] + i4[3]);
    cx<TC> *c = C + (int64_t)j * ldc + i;
    if (beta != 0.0) {
        re = alpha * re + beta * (double)c->re;
        im = alpha * im + beta * (double)c->im;
    } else {
        re *= alpha;
        im *= alpha;
    }
    *c = cx<TC>{(TC)re, (TC)im};
}

// P[j][i] = sum_s part[s][j][i]; Q[j][i] = sum_t D_blk(i)[i - lo][t] P[j][lo + t]
// One work-group per band j. The splits are divided among G thread groups
// (G M <= blockDim.x), each thread summing its splits in four independent
// chains; the group sums are added in a fixed order, so the result does not
// depend on timing. P of the band is then in LDS for the D blocks.
constexpr int kRedThreads = 1024, kRedMaxGroups = 8;
__host__ __device__ inline int reduce_groups(int M) {
    return M <= 0 ? 1 : std::max(1, std::min(kRedMaxGroups, std::min(kRedThreads / M, 4096 / M)));
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_reduce_dapply(int M, int nsplit, const cx<T> *__restrict__ part,
                                                               int N, const double *__restrict__ dmat,
                                                               const int *__restrict__ blo, const int *__restrict__ bn,
                                                               const int *__restrict__ bdoff, cx<T> *__restrict__ P,
                                                               cx<T> *__restrict__ Q) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<double> *pl = reinterpret_cast<cx<double> *>(smem);   // [G][M] group sums, then the total in [0][M]
    const int j = blockIdx.x;
    const int G = reduce_groups(M);
    const int64_t sstride = (int64_t)N * M;
    for (int idx = threadIdx.x; idx < G * M; idx += blockDim.x) {
        const int g = idx / M, i = idx - g * M;
        const cx<T> *src = part + (int64_t)j * M + i;
        double re[4] = {0.0, 0.0, 0.0, 0.0}, im[4] = {0.0, 0.0, 0.0, 0.0};
        int s = g;
        for (; s + 3 * G < nsplit; s += 4 * G) {
            cx<T> v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = src[(int64_t)(s + u * G) * sstride];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                re[u] += (double)v[u].re;
                im[u] += (double)v[u].im;
            }
        }
        for (int u = 0; s < nsplit; s += G, ++u) {
            const cx<T> v = src[(int64_t)s * sstride];
            re[u] += (double)v.re;
            im[u] += (double)v.im;
        }
        pl[idx] = cx<double>{(re[0] + re[1]) + (re[2] + re[3]), (im[0] + im[1]) + (im[2] + im[3])};
    }
    __syncthreads();
    for (int i = threadIdx.x; i < M; i += blockDim.x) {
        cx<double> t = pl[i];
        for (int g = 1; g < G; ++g) t = t + pl[g * M + i];
        pl[i] = t;
        if (P) P[(int64_t)j * M + i] = cx<T>{(T)t.re, (T)t.im};
    }
    __syncthreads();
    for (int i = threadIdx.x; i < M; i += blockDim.x) {
        const int lo = blo[i], n = bn[i];
        const double *d = dmat + bdoff[i] + (int64_t)(i - lo) * n;
        double re = 0.0, im = 0.0;
        for (int t = 0; t < n; ++t) {
            re += d[t] * pl[lo + t].re;
            im += d[t] * pl[lo + t].im;
        }
        Q[(int64_t)j * M + i] = cx<T>{(T)re, (T)im};
    }
}

// ----------------------------------------------------------------- NN ------
// C[j][g] = alpha * sum_i A[j][i] B[i][g] + beta * C[j][g]
// TS is the type A and B are stored in; they are rounded to T while staged.
template <typename T, typename TC, typename TS = T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kGemmWaves))) void k_gemm_nn(int M, int G, int K, const cx<TS> *__restrict__ A, int64_t lda,
                                                 const cx<TS> *__restrict__ B, int64_t ldb, cx<TC> *__restrict__ C,
                                                 int64_t ldc, double alpha, double beta) {
    __shared__ cx<T> As[TM][KP];
    __shared__ cx<T> Bs[KT][TN + 1];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int bx, by, bz;
    xcd_block(bx, by, bz);   // the row tiles of one column block share an L2
    const int j0 = bx * TM, g0 = by * TN;
    using AV = typename Acc<T>::V;
    AV c1[2][2], c2[2][2], c3[2][2];   // sums of ar br, ai bi, (ar + ai)(br + bi)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) c1[a][b] = c2[a][b] = c3[a][b] = Acc<T>::zero();
    const int wj = (w & 1) * 32, wg = (w >> 1) * 32;
    const int ar = tid >> 2, ak = (tid & 3) * 4;       // A loader: row j, 4 consecutive i
    const int bk = tid >> 4, bg = (tid & 15) * 4;      // B loader: row i, 4 consecutive g
    cx<T> ra[4], rb[4];
    auto load = [&](int k0) {
        const int gj = j0 + ar;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int gk = k0 + ak + q;
            ra[q] = (gj < M && gk < K) ? cvt<T>(A[gj * lda + gk]) : cx<T>{T(0), T(0)};
        }
        const int gk = k0 + bk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int gg = g0 + bg + q;
            rb[q] = (gk < K && gg < G) ? cvt<T>(B[gk * ldb + gg]) : cx<T>{T(0), T(0)};
        }
    };
    load(0);
    for (int k0 = 0; k0 < K; k0 += KT) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[ar][ak + q] = ra[q];
            Bs[bk][bg + q] = rb[q];
        }
        __syncthreads();
        if (k0 + KT < K) load(k0 + KT);   // next stage in flight while this one multiplies
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kk = 4 * q + (lane >> 4);
            cx<T> a[2], b[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) a[r] = As[wj + 16 * r + (lane & 15)][kk];
#pragma unroll
            for (int c = 0; c < 2; ++c) b[c] = Bs[kk][wg + 16 * c + (lane & 15)];
            T as[2], bs[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) as[r] = a[r].re + a[r].im;
#pragma unroll
            for (int c = 0; c < 2; ++c) bs[c] = b[c].re + b[c].im;
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    // a b with three real products:
                    //   re = ar br - ai bi,  im = (ar + ai)(br + bi) - ar br - ai bi
                    c1[r][c] = Acc<T>::mma(a[r].re, b[c].re, c1[r][c]);
                    c2[r][c] = Acc<T>::mma(a[r].im, b[c].im, c2[r][c]);
                    c3[r][c] = Acc<T>::mma(as[r], bs[c], c3[r][c]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int gg = g0 + wg + 16 * c + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gj = j0 + wj + 16 * r + Acc<T>::row(lane, e);
                if (gj < M && gg < G) {
                    cx<TC> *p = C + (int64_t)gj * ldc + gg;
                    const double p1 = c1[r][c][e], p2 = c2[r][c][e], p3 = c3[r][c][e];
                    double re = alpha * (p1 - p2), im = alpha * (p3 - p1 - p2);
                    if (beta != 0.0) {
                        const cx<TC> o = *p;
                        re += beta * (double)o.re;
                        im += beta * (double)o.im;
                    }
                    *p = cx<TC>{(TC)re, (TC)im};
                }
            }
        }
}

// grad_d[blk(i)][i - lo][t] (+)= sum_n Re(Q[n][i] conj(P[n][lo + t])), one thread per projector i.
template <typename T>
__global__ void k_grad_d(int nb, int M, const cx<T> *__restrict__ P, const cx<T> *__restrict__ Q,
                         const int *__restrict__ blo, const int *__restrict__ bn, const int *__restrict__ bdoff,
                         double *__restrict__ gd, int first) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int lo = blo[i], n = bn[i];
    double *out = gd + bdoff[i] + (int64_t)(i - lo) * n;
    for (int t = 0; t < n; ++t) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) {
            const cx<T> q = Q[(int64_t)b * M + i], p = P[(int64_t)b * M + lo + t];
            s += (double)q.re * (double)p.re + (double)q.im * (double)p.im;
        }
        out[t] = first ? s : out[t] + s;
    }
}

// ------------------------------------------------------------ launchers ----
// Default K chunk: at least 512 work-groups, chunks of at most 1024 (a K chunk of
// A and B read by every tile of the chunk stays in the caches, where one long K
// range per tile streams A once per column of tiles from HBM: at 2304 x 1024 x
// 161,235 the projection read 13.7x its operands with one split, measured with
// FETCH_SIZE), but no more splits than keep the partial sums under kPartCap bytes.
constexpr size_t kPartCap = size_t(1) << 30;
static int splits_for(int M, int N, int K, int chunk_hint, int *chunk) {
    const int tiles = ceil_div(M, TM) * ceil_div(N, TN);
    int c = chunk_hint > 0 ? chunk_hint : 0;
    if (c <= 0) {
        const int want = std::max(1, 512 / std::max(1, tiles));
        c = std::min(1024, std::max(256, ceil_div(K, want)));
        const int64_t max_splits = std::max<int64_t>(1, (int64_t)(kPartCap / ((size_t)M * N * 16)));
        c = std::max<int64_t>(c, ceil_div64(K, max_splits));
    }
    c = ceil_div(c, KT) * KT;
    *chunk = c;
    return std::max(1, ceil_div(K, c));
}

// Upper bound over every K' <= K: the split count grows with K up to the cap (with
// a chunk hint without one).
size_t gemm_cn_part_bytes(int M, int N, int K, int elem_bytes, int chunk_hint) {
    int c;
    int ns = splits_for(M, N, K, chunk_hint, &c);
    if (chunk_hint <= 0) ns = std::max(ns, std::max(1, 512 / std::max(1, ceil_div(M, TM) * ceil_div(N, TN))));
    return (size_t)ns * M * N * elem_bytes;
}

template <typename T, typename TS = T>
static int cn_part(int M, int N, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *part,
                   int chunk_hint, int *nsplit, hipStream_t st) {
    int chunk;
    const int ns = splits_for(M, N, K, chunk_hint, &chunk);
    *nsplit = ns;
    dim3 grid(ceil_div(M, TM), ceil_div(N, TN), ns);
    // group of row tiles: about one XCD's resident work-groups (32 CUs x 3) per group;
    // a chunk of at most two such groups keeps the row tiles fastest (one group): at
    // 864 x 512 per k-point that order measured 1-2% faster than groups of 12 rows
    const int tiles = (int)(grid.x * grid.y);
    const int gm = tiles <= 192 ? (int)grid.x : std::max(1, std::min((int)grid.x, 96 / (int)grid.y));
    KernelTimer kt("gemm_cn", st);
    hipLaunchKernelGGL((k_gemm_cn_part<T, TS>), grid, dim3(256), 0, st, M, N, K, chunk, static_cast<const cx<TS> *>(A),
                       lda, static_cast<const cx<TS> *>(B), ldb, static_cast<cx<T> *>(part), gm);
    return check_launch("gemm_cn");
}

// T: arithmetic and partial sums; TS: storage of A, B and C.
template <typename T, typename TS = T>
static int gemm_cn_t(int M, int N, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
                     int64_t ldc, double alpha, double beta, void *part, int chunk_hint, hipStream_t st) {
    if (M <= 0 || N <= 0) return ABACUS_PW_OK;
    int ns;
    APW_TRY((cn_part<T, TS>(M, N, K, A, lda, B, ldb, part, chunk_hint, &ns, st)));
    const int64_t tot = (int64_t)M * N;
    KernelTimer kt("gemm_reduce", st);
    hipLaunchKernelGGL((k_reduce<T, TS>), dim3((unsigned)ceil_div64(tot, 256)), dim3(256), 0, st, M, N, ns,
                       static_cast<const cx<T> *>(part), static_cast<cx<TS> *>(C), ldc, alpha, beta);
    return check_launch("gemm_reduce");
}

int reduce_parts_f32_to_f64(int M, int N, int nsplit, const void *part, void *C, int64_t ldc, double alpha,
                            double beta, hipStream_t st) {
    if (M <= 0 || N <= 0) return ABACUS_PW_OK;
    const int64_t tot = (int64_t)M * N;
    KernelTimer kt("gemm_reduce", st);
    hipLaunchKernelGGL((k_reduce<float, double>), dim3((unsigned)ceil_div64(tot, 256)), dim3(256), 0, st, M, N, nsplit,
                       static_cast<const c32 *>(part), static_cast<z64 *>(C), ldc, alpha, beta);
    return check_launch("gemm_reduce");
}

int gemm_cn_f32_of_f64(int M, int N, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
                       int64_t ldc, double alpha, double beta, void *part, int chunk_hint, hipStream_t st) {
    return gemm_cn_t<float, double>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, part, chunk_hint, st);
}

int gemm_cn(int prec, int M, int N, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
            int64_t ldc, double alpha, double beta, void *part, int chunk_hint, hipStream_t st) {
    return prec == 0 ? gemm_cn_t<double>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, part, chunk_hint, st)
                     : gemm_cn_t<float>(M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, part, chunk_hint, st);
}

template <typename T>
static int proj_dapply_t(int M, int N, int K, const void *Bm, int64_t ldb, const void *psi, int64_t ldp,
                         const double *dmat, const int *blo, const int *bn, const int *bdoff, void *P, void *Q,
                         void *part, int chunk_hint, hipStream_t st) {
    if (M <= 0 || N <= 0) return ABACUS_PW_OK;
    int ns;
    APW_TRY(cn_part<T>(M, N, K, Bm, ldb, psi, ldp, part, chunk_hint, &ns, st));
    const size_t lds = (size_t)reduce_groups(M) * M * sizeof(cx<double>);
    if (lds > 64 * 1024) return set_error(ABACUS_PW_EBAD_SHAPE, "too many projectors for the D-apply stage");
    KernelTimer kt("reduce_dapply", st);
    hipLaunchKernelGGL(k_reduce_dapply<T>, dim3(N), dim3(kRedThreads), lds, st, M, ns, static_cast<const cx<T> *>(part), N,
                       dmat, blo, bn, bdoff, static_cast<cx<T> *>(P), static_cast<cx<T> *>(Q));
    return check_launch("reduce_dapply");
}

int proj_dapply(int prec, int M, int N, int K, const void *Bm, int64_t ldb, const void *psi, int64_t ldp,
                const double *dmat, const int *blo, const int *bn, const int *bdoff, void *P, void *Q, void *part,
                int chunk_hint, hipStream_t st) {
    return prec == 0 ? proj_dapply_t<double>(M, N, K, Bm, ldb, psi, ldp, dmat, blo, bn, bdoff, P, Q, part,
                                             chunk_hint, st)
                     : proj_dapply_t<float>(M, N, K, Bm, ldb, psi, ldp, dmat, blo, bn, bdoff, P, Q, part,
                                            chunk_hint, st);
}

template <typename T, typename TC, typename TS = T>
static int gemm_nn_t(int M, int G, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
                     int64_t ldc, double alpha, double beta, hipStream_t st) {
    if (M <= 0 || G <= 0) return ABACUS_PW_OK;
    dim3 grid(ceil_div(M, TM), ceil_div(G, TN));
    KernelTimer kt("gemm_nn", st);
    hipLaunchKernelGGL((k_gemm_nn<T, TC, TS>), grid, dim3(256), 0, st, M, G, K, static_cast<const cx<TS> *>(A), lda,
                       static_cast<const cx<TS> *>(B), ldb, static_cast<cx<TC> *>(C), ldc, alpha, beta);
    return check_launch("gemm_nn");
}

int gemm_nn_f32_of_f64(int M, int G, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
                       int64_t ldc, double alpha, double beta, hipStream_t st) {
    return gemm_nn_t<float, double, double>(M, G, K, A, lda, B, ldb, C, ldc, alpha, beta, st);
}

int gemm_nn(int prec, int M, int G, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
            int64_t ldc, double alpha, double beta, hipStream_t st) {
    return prec == 0 ? gemm_nn_t<double, double>(M, G, K, A, lda, B, ldb, C, ldc, alpha, beta, st)
                     : gemm_nn_t<float, float>(M, G, K, A, lda, B, ldb, C, ldc, alpha, beta, st);
}

int gemm_nn_f32_into_f64(int M, int G, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
                         int64_t ldc, double alpha, double beta, hipStream_t st) {
    return gemm_nn_t<float, double>(M, G, K, A, lda, B, ldb, C, ldc, alpha, beta, st);
}

int reduce_dapply_f32(int M, int N, int nsplit, const void *part, const double *dmat, const int *blo, const int *bn,
                      const int *bdoff, void *Q, hipStream_t st) {
    const size_t lds = (size_t)reduce_groups(M) * M * sizeof(cx<double>);
    if (lds > 64 * 1024) return set_error(ABACUS_PW_EBAD_SHAPE, "too many projectors for the D-apply stage");
    KernelTimer kt("reduce_dapply", st);
    hipLaunchKernelGGL(k_reduce_dapply<float>, dim3(N), dim3(kRedThreads), lds, st, M, nsplit, static_cast<const c32 *>(part),
                       N, dmat, blo, bn, bdoff, static_cast<c32 *>(nullptr), static_cast<c32 *>(Q));
    return check_launch("reduce_dapply");
}

int grad_d_accumulate(int prec, int nb, int M, const void *P, const void *Q, const int *blo, const int *bn,
                      const int *bdoff, double *gd, int first, hipStream_t st) {
    KernelTimer kt("grad_d", st);
    if (prec == 0)
        hipLaunchKernelGGL(k_grad_d<double>, dim3(ceil_div(M, 64)), dim3(64), 0, st, nb, M,
                           static_cast<const z64 *>(P), static_cast<const z64 *>(Q), blo, bn, bdoff, gd, first);
    else
        hipLaunchKernelGGL(k_grad_d<float>, dim3(ceil_div(M, 64)), dim3(64), 0, st, nb, M,
                           static_cast<const c32 *>(P), static_cast<const c32 *>(Q), blo, bn, bdoff, gd, first);
    return check_launch("grad_d");
}

}  // namespace apw

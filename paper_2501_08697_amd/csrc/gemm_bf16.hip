// Projector GEMMs of the Kleinman-Bylander term (Sec. II.A) with BF16
// operands and FP32 accumulation on v_mfma_f32_16x16x32_bf16 (gfx950), for the
// MIXED_BF16 mode:
//
//   CN  part[s][j][i] = sum_{k in split s} conj(A[i][k]) B[j][k]
//       A: beta as packed complex bf16 (re in the low half-word), B: psi as
//       complex128 or complex64, rounded to bf16 while it is staged in LDS.
//   NN  C[j][g] += sum_i A[j][i] B[i][g]
//       A: Q = D P as complex64 (rounded to bf16 in LDS), B: beta packed bf16,
//       C: complex128 H psi.
//
// The instruction takes eight consecutive k of A and of B per lane (A[i][k]
// at lane i + 16 (k / 8), B[k][j] at lane j + 16 (k / 8)) and returns D[i][j]
// at lane j + 16 (i / 4), element i % 4, like the FP32 16x16x4 form.
// Rounding to bf16 is round-to-nearest-even on the FP32 value.
#include "common.hpp"
#include "gemm.hpp"

namespace apw {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint32_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ uint32_t pack_bf16(float re, float im) { return bf16_bits(re) | (bf16_bits(im) << 16); }

template <typename T> __device__ __forceinline__ uint32_t pack_c(cx<T> v) {
    return pack_bf16(static_cast<float>(v.re), static_cast<float>(v.im));
}

// Split 8 packed complex bf16 values into real and imaginary bf16 vectors.
__device__ __forceinline__ void unpack8(const uint32_t *p, bf8 &re, bf8 &im, bool neg_im) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const unsigned short r = (unsigned short)(p[t] & 0xFFFFu);
        unsigned short i = (unsigned short)(p[t] >> 16);
        if (neg_im) i ^= 0x8000u;
        re[t] = __builtin_bit_cast(__bf16, r);
        im[t] = __builtin_bit_cast(__bf16, i);
    }
}

__device__ __forceinline__ f4 mma(bf8 a, bf8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

constexpr int BT = 64, BK = 32, BKP = BK + 4;   // tile, k per stage, padded LDS row (16-byte aligned)

template <typename TB>
__global__ __launch_bounds__(256) void k_cn_bf16(int M, int N, int K, int kchunk, const uint32_t *__restrict__ A,
                                                 int64_t lda, const cx<TB> *__restrict__ B, int64_t ldb,
                                                 c32 *__restrict__ part) {
    __shared__ __align__(16) uint32_t As[BT][BKP];
    __shared__ __align__(16) uint32_t Bs[BT][BKP];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int bx, by, bz;
    xcd_block(bx, by, bz);
    const int i0 = bx * BT, j0 = by * BT, s = bz;
    const int kb = s * kchunk, ke = min(K, kb + kchunk);
    f4 cre[2][2], cim[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) cre[a][b] = cim[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    const int lr = tid >> 2, lk = (tid & 3) * 8;   // loader: row, first of 8 k
    const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
    const int gi = i0 + lr, gj = j0 + lr;
    for (int k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int gk = k0 + lk + q;
            As[lr][lk + q] = (gi < M && gk < ke) ? A[gi * lda + gk] : 0u;
            Bs[lr][lk + q] = (gj < N && gk < ke) ? pack_c(B[gj * ldb + gk]) : 0u;
        }
        __syncthreads();
        const int kk = 8 * (lane >> 4);
        bf8 are[2], aim[2], bre[2], bim[2], naim[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            unpack8(&As[wi + 16 * r + (lane & 15)][kk], are[r], aim[r], false);
            bf8 tmp;
            unpack8(&As[wi + 16 * r + (lane & 15)][kk], tmp, naim[r], true);
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) unpack8(&Bs[wj + 16 * c + (lane & 15)][kk], bre[c], bim[c], false);
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                // conj(a) b = (ar br + ai bi) + i (ar bi - ai br)
                cre[r][c] = mma(are[r], bre[c], cre[r][c]);
                cre[r][c] = mma(aim[r], bim[c], cre[r][c]);
                cim[r][c] = mma(are[r], bim[c], cim[r][c]);
                cim[r][c] = mma(naim[r], bre[c], cim[r][c]);
            }
        __syncthreads();
    }
    c32 *out = part + (int64_t)s * N * M;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int jj = j0 + wj + 16 * c + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int ii = i0 + wi + 16 * r + 4 * (lane >> 4) + e;
                if (ii < M && jj < N) out[(int64_t)jj * M + ii] = c32{cre[r][c][e], cim[r][c][e]};
            }
        }
}

// C[j][g] += sum_i A[j][i] B[i][g]; A complex64 [M][lda], B packed bf16 [K][ldb], C complex128.
__global__ __launch_bounds__(256) void k_nn_bf16(int M, int G, int K, const c32 *__restrict__ A, int64_t lda,
                                                 const uint32_t *__restrict__ B, int64_t ldb, z64 *__restrict__ C,
                                                 int64_t ldc) {
    __shared__ __align__(16) uint32_t As[BT][BKP];    // [j][i]
    __shared__ __align__(16) uint32_t Bt[BT][BKP];    // transposed: [g][i]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int bx, by, bz;
    xcd_block(bx, by, bz);
    const int j0 = bx * BT, g0 = by * BT;
    f4 cre[2][2], cim[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) cre[a][b] = cim[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    const int wj = (w & 1) * 32, wg = (w >> 1) * 32;
    const int ar = tid >> 2, ak = (tid & 3) * 8;      // A loader: row j, 8 consecutive i
    const int bk = tid >> 3, bg = (tid & 7) * 8;      // B loader: row i, 8 consecutive g
    for (int k0 = 0; k0 < K; k0 += BK) {
        {
            const int gj = j0 + ar;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int gk = k0 + ak + q;
                As[ar][ak + q] = (gj < M && gk < K) ? pack_c(A[gj * lda + gk]) : 0u;
            }
            const int gk = k0 + bk;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int gg = g0 + bg + q;
                Bt[bg + q][bk] = (gk < K && gg < G) ? B[gk * ldb + gg] : 0u;
            }
        }
        __syncthreads();
        const int kk = 8 * (lane >> 4);
        bf8 are[2], aim[2], naim[2], bre[2], bim[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            unpack8(&As[wj + 16 * r + (lane & 15)][kk], are[r], aim[r], false);
            bf8 tmp;
            unpack8(&As[wj + 16 * r + (lane & 15)][kk], tmp, naim[r], true);
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) unpack8(&Bt[wg + 16 * c + (lane & 15)][kk], bre[c], bim[c], false);
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                // a b = (ar br - ai bi) + i (ar bi + ai br)
                cre[r][c] = mma(are[r], bre[c], cre[r][c]);
                cre[r][c] = mma(naim[r], bim[c], cre[r][c]);
                cim[r][c] = mma(are[r], bim[c], cim[r][c]);
                cim[r][c] = mma(aim[r], bre[c], cim[r][c]);
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
                const int gj = j0 + wj + 16 * r + 4 * (lane >> 4) + e;
                if (gj < M && gg < G) {
                    z64 *p = C + (int64_t)gj * ldc + gg;
                    *p = z64{p->re + (double)cre[r][c][e], p->im + (double)cim[r][c][e]};
                }
            }
        }
}

// packed bf16 copy of a complex128 array
__global__ void k_pack_bf16(int64_t n, const z64 *__restrict__ in, uint32_t *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = pack_c(in[i]);
}

// ------------------------------------------------------------ launchers ----
int pack_bf16(int64_t n, const void *in, void *out, hipStream_t st) {
    int64_t blocks = std::min<int64_t>(ceil_div64(n, 256), 65536);
    KernelTimer kt("convert", st);
    hipLaunchKernelGGL(k_pack_bf16, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, n,
                       static_cast<const z64 *>(in), static_cast<uint32_t *>(out));
    return check_launch("pack_bf16");
}

size_t gemm_cn_bf16_part_bytes(int M, int N, int K, int chunk_hint) {
    const int tiles = ceil_div(M, BT) * ceil_div(N, BT);
    int c = chunk_hint > 0 ? ceil_div(chunk_hint, BK) * BK : 0;
    int ns = c > 0 ? ceil_div(K, c) : std::max(1, 512 / std::max(1, tiles));
    return (size_t)std::max(ns, 1) * M * N * sizeof(c32) + 256;
}

int proj_dapply_bf16(int M, int N, int K, const void *Bpk, int64_t ldb, const void *psi, int psi_is_f64, int64_t ldp,
                     const double *dmat, const int *blo, const int *bn, const int *bdoff, void *Q, void *part,
                     int chunk_hint, hipStream_t st) {
    if (M <= 0 || N <= 0) return ABACUS_PW_OK;
    const int tiles = ceil_div(M, BT) * ceil_div(N, BT);
    int c = chunk_hint > 0 ? chunk_hint : std::max(512, ceil_div(K, std::max(1, 512 / std::max(1, tiles))));
    c = ceil_div(c, BK) * BK;
    const int ns = std::max(1, ceil_div(K, c));
    dim3 grid(ceil_div(M, BT), ceil_div(N, BT), ns);
    {
        KernelTimer kt("gemm_cn_bf16", st);
        if (psi_is_f64)
            hipLaunchKernelGGL(k_cn_bf16<double>, grid, dim3(256), 0, st, M, N, K, c,
                               static_cast<const uint32_t *>(Bpk), ldb, static_cast<const z64 *>(psi), ldp,
                               static_cast<c32 *>(part));
        else
            hipLaunchKernelGGL(k_cn_bf16<float>, grid, dim3(256), 0, st, M, N, K, c,
                               static_cast<const uint32_t *>(Bpk), ldb, static_cast<const c32 *>(psi), ldp,
                               static_cast<c32 *>(part));
        APW_TRY(check_launch("gemm_cn_bf16"));
    }
    return reduce_dapply_f32(M, N, ns, part, dmat, blo, bn, bdoff, Q, st);
}

int gemm_nn_bf16_into_f64(int M, int G, int K, const void *A, int64_t lda, const void *Bpk, int64_t ldb, void *C,
                          int64_t ldc, hipStream_t st) {
    if (M <= 0 || G <= 0) return ABACUS_PW_OK;
    dim3 grid(ceil_div(M, BT), ceil_div(G, BT));
    KernelTimer kt("gemm_nn_bf16", st);
    hipLaunchKernelGGL(k_nn_bf16, grid, dim3(256), 0, st, M, G, K, static_cast<const c32 *>(A), lda,
                       static_cast<const uint32_t *>(Bpk), ldb, static_cast<z64 *>(C), ldc);
    return check_launch("gemm_nn_bf16");
}

}  // namespace apw

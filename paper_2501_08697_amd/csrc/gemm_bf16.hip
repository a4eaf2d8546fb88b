// Projector GEMMs of the Kleinman-Bylander term (Sec. II.A) with BF16
// operands and FP32 accumulation on v_mfma_f32_16x16x32_bf16 (gfx950), for the
// MIXED_BF16 mode:
//
//   CN  part[s][j][i] = sum_{k in split s} conj(A[i][k]) B[j][k]
//       A: beta, B: psi, both as packed complex bf16 (re in the low half-word)
//       rows padded with zeros to a multiple of 32.
//   NN  C[j][g] += sum_i Q[j][i] beta[i][g]
//       Q = D P and the transposed beta [g][i], both packed bf16 with the
//       projector index padded to a multiple of 32; C: complex128 H psi.
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

__device__ __forceinline__ f4 mma(bf8 a, bf8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }


// ---------------------------------------------------------------------------
// CN with 128 x 128 work-group tiles. Both operands are packed bf16 rows whose
// leading dimension is a multiple of 32 and whose padding is zero, so every
// stage of 32 k is a set of aligned 16-byte loads with no bounds on k. The
// loaders split each packed pair into planar real and imaginary bf16 rows in
// LDS (v_perm), so a lane's MFMA fragment (eight consecutive k of one row) is
// one 16-byte LDS read. Each wave owns a 64 x 64 quarter: 4 x 4 tiles of
// 16 x 16, four MFMAs per tile per stage (conj(a) b). The next stage's global
// values are fetched into registers while the current stage computes.
// ---------------------------------------------------------------------------
constexpr int T2 = 128;           // work-group tile (rows of A and of B)
constexpr int BK2 = 32;           // k per stage
constexpr int P2 = 20;            // LDS row pitch in 32-bit words (16 bf16 pairs + 4 pad; 80 bytes)

typedef unsigned int u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf8 as_bf8(u4 v) { return __builtin_bit_cast(bf8, v); }

// 16 packed pairs (re low, im high) -> 8 words of real pairs and 8 words of imaginary pairs
__device__ __forceinline__ void split16(const u4 g[4], u4 re[2], u4 im[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const u4 a = g[2 * h], b = g[2 * h + 1];
        re[h] = u4{__builtin_amdgcn_perm(a.y, a.x, 0x05040100u), __builtin_amdgcn_perm(a.w, a.z, 0x05040100u),
                   __builtin_amdgcn_perm(b.y, b.x, 0x05040100u), __builtin_amdgcn_perm(b.w, b.z, 0x05040100u)};
        im[h] = u4{__builtin_amdgcn_perm(a.y, a.x, 0x07060302u), __builtin_amdgcn_perm(a.w, a.z, 0x07060302u),
                   __builtin_amdgcn_perm(b.y, b.x, 0x07060302u), __builtin_amdgcn_perm(b.w, b.z, 0x07060302u)};
    }
}

// S[j][i] = sum_{k in split s} op(A[i][k]) B[j][k], op = conj when kConj; A [M][lda], B [N][ldb]
// packed bf16, lda, ldb, kchunk and the K range multiples of 32 (zero beyond the data).
// kIntoF64: out is complex128 C with C[j][i] += S[j][i] (ldo), one split; else out is
// complex64 part[s][j][i] (column-major M x N per split).
template <bool kConj, bool kIntoF64>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_bf16_t128(int M, int N, int Kp, int kchunk, const uint32_t *__restrict__ A,
                                                   int64_t lda, const uint32_t *__restrict__ B, int64_t ldb,
                                                   void *__restrict__ out, int64_t ldo, int b_fastest) {
    __shared__ __align__(16) uint32_t Are[T2 * P2], Aim[T2 * P2], Bre[T2 * P2], Bim[T2 * P2];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int bx, by, bz;
    xcd_block(bx, by, bz);
    // b_fastest: the grid's x runs over B tiles, so the blocks that share an A tile run together
    const int i0 = (b_fastest ? by : bx) * T2, j0 = (b_fastest ? bx : by) * T2, s = bz;
    const int kb = s * kchunk, ke = min(Kp, kb + kchunk);
    // loader: row tid / 2 of each tile, k half (tid % 2) * 16 of the stage
    const int lr = tid >> 1, lh = (tid & 1) * 16;
    const bool arow = i0 + lr < M, brow = j0 + lr < N;
    // a loader row past M (N) reads row 0 instead: such a row only feeds outputs with
    // i >= M (j >= N), which are never stored, and the loads need no per-row branch
    const uint32_t *ga = A + (int64_t)(arow ? i0 + lr : 0) * lda + lh;
    const uint32_t *gb = B + (int64_t)(brow ? j0 + lr : 0) * ldb + lh;
    u4 pa[4], pb[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            pa[q] = *reinterpret_cast<const u4 *>(ga + k0 + 4 * q);
            pb[q] = *reinterpret_cast<const u4 *>(gb + k0 + 4 * q);
        }
    };
    f4 cre[4][4], cim[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) cre[r][c] = cim[r][c] = f4{0.f, 0.f, 0.f, 0.f};
    const int wi = (w & 1) * 64, wj = (w >> 1) * 64;
    const int fr = lane & 15, fk = 4 * (lane >> 4);   // fragment row and word offset (8 bf16 = 4 words)
    if (kb < ke) fetch(kb);
    for (int k0 = kb; k0 < ke; k0 += BK2) {
        {
            u4 re[2], im[2];
            split16(pa, re, im);
            const int o = lr * P2 + lh / 2;
            *reinterpret_cast<u4 *>(&Are[o]) = re[0];
            *reinterpret_cast<u4 *>(&Are[o + 4]) = re[1];
            *reinterpret_cast<u4 *>(&Aim[o]) = im[0];
            *reinterpret_cast<u4 *>(&Aim[o + 4]) = im[1];
            split16(pb, re, im);
            *reinterpret_cast<u4 *>(&Bre[o]) = re[0];
            *reinterpret_cast<u4 *>(&Bre[o + 4]) = re[1];
            *reinterpret_cast<u4 *>(&Bim[o]) = im[0];
            *reinterpret_cast<u4 *>(&Bim[o + 4]) = im[1];
        }
        // the next stage's loads, in flight while this stage computes, go out before the
        // barrier, so that the wait for the other waves' LDS writes also covers their latency
        // (at 1024 bands x 161k PW x 2304 projectors: accumulation 4.96 -> 4.74 ms, projection
        // 3.39 -> 3.34 ms)
        if (k0 + BK2 < ke) fetch(k0 + BK2);
        __syncthreads();
        bf8 br[4], bi[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int o = (wj + 16 * c + fr) * P2 + fk;
            br[c] = as_bf8(*reinterpret_cast<const u4 *>(&Bre[o]));
            bi[c] = as_bf8(*reinterpret_cast<const u4 *>(&Bim[o]));
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = (wi + 16 * r + fr) * P2 + fk;
            const u4 ar4 = *reinterpret_cast<const u4 *>(&Are[o]);
            const u4 ai4 = *reinterpret_cast<const u4 *>(&Aim[o]);
            const bf8 ar = as_bf8(ar4), ai = as_bf8(ai4), nai = as_bf8(ai4 ^ u4{0x80008000u, 0x80008000u,
                                                                              0x80008000u, 0x80008000u});
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                // conj(a) b = (ar br + ai bi) + i (ar bi - ai br);  a b = (ar br - ai bi) + i (ar bi + ai br)
                cre[r][c] = mma(ar, br[c], cre[r][c]);
                cre[r][c] = mma(kConj ? ai : nai, bi[c], cre[r][c]);
                cim[r][c] = mma(ar, bi[c], cim[r][c]);
                cim[r][c] = mma(kConj ? nai : ai, br[c], cim[r][c]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int jj = j0 + wj + 16 * c + fr;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int ii = i0 + wi + 16 * r + 4 * (lane >> 4) + e;
                if (ii < M && jj < N) {
                    if (kIntoF64) {
                        z64 *p = static_cast<z64 *>(out) + (int64_t)jj * ldo + ii;
                        *p = z64{p->re + (double)cre[r][c][e], p->im + (double)cim[r][c][e]};
                    } else {
                        static_cast<c32 *>(out)[(int64_t)s * N * M + (int64_t)jj * M + ii] =
                            c32{cre[r][c][e], cim[r][c][e]};
                    }
                }
            }
        }
}

// packed bf16 copy of rows [rows][K] (leading dimension ldi) into [rows][ldo], zero for K <= c < ldo
template <typename T>
__global__ void k_pack_bf16_rows(int rows, int K, const cx<T> *__restrict__ in, int64_t ldi,
                                 uint32_t *__restrict__ out, int64_t ldo) {
    const int64_t n = (int64_t)rows * ldo;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / ldo;
        const int c = (int)(e - r * ldo);
        out[e] = c < K ? pack_c(in[r * ldi + c]) : 0u;
    }
}

// out[g][i] = packed bf16 of in[i][g] for i < rows, 0 for rows <= i < ldo (in: complex128 [rows][ldi],
// g < cols): 32 x 64 tiles through LDS so that reads and writes are both row-contiguous.
__global__ __launch_bounds__(256) void k_pack_bf16_transpose(int rows, int cols, const z64 *__restrict__ in,
                                                              int64_t ldi, uint32_t *__restrict__ out, int64_t ldo) {
    __shared__ uint32_t t[32][64 + 1];
    const int i0 = blockIdx.y * 32, g0 = blockIdx.x * 64;
    for (int e = threadIdx.x; e < 32 * 64; e += blockDim.x) {
        const int r = e / 64, c = e % 64;
        const int i = i0 + r, g = g0 + c;
        t[r][c] = (i < rows && g < cols) ? pack_c(in[(int64_t)i * ldi + g]) : 0u;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * 64; e += blockDim.x) {
        const int c = e / 32, r = e % 32;
        const int i = i0 + r, g = g0 + c;
        if (g < cols && i < ldo) out[(int64_t)g * ldo + i] = t[r][c];
    }
}

// ------------------------------------------------------------ launchers ----
int pack_bf16_transpose(int rows, int cols, const void *in, int64_t ldi, void *out, int64_t ldo, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return ABACUS_PW_OK;
    KernelTimer kt("convert", st);
    hipLaunchKernelGGL(k_pack_bf16_transpose, dim3(ceil_div(cols, 64), ceil_div((int)ldo, 32)), dim3(256), 0, st,
                       rows, cols, static_cast<const z64 *>(in), ldi, static_cast<uint32_t *>(out), ldo);
    return check_launch("pack_bf16_transpose");
}

int pack_bf16_rows(int rows, int K, const void *in, int in_is_f64, int64_t ldi, void *out, int64_t ldo,
                   hipStream_t st) {
    if (rows <= 0) return ABACUS_PW_OK;
    const int64_t blocks = std::min<int64_t>(ceil_div64((int64_t)rows * ldo, 256), 65536);
    KernelTimer kt("convert", st);
    if (in_is_f64)
        hipLaunchKernelGGL(k_pack_bf16_rows<double>, dim3((unsigned)blocks), dim3(256), 0, st, rows, K,
                           static_cast<const z64 *>(in), ldi, static_cast<uint32_t *>(out), ldo);
    else
        hipLaunchKernelGGL(k_pack_bf16_rows<float>, dim3((unsigned)blocks), dim3(256), 0, st, rows, K,
                           static_cast<const c32 *>(in), ldi, static_cast<uint32_t *>(out), ldo);
    return check_launch("pack_bf16_rows");
}

// splits of the CN product: enough work-groups to fill the chip (>= 1024), stages of at least 512 k
static int cn_bf16_chunk(int M, int N, int Kp, int chunk_hint) {
    if (chunk_hint > 0) return ceil_div(chunk_hint, BK2) * BK2;
    const int tiles = ceil_div(M, T2) * ceil_div(N, T2);
    const int want = std::max(1, ceil_div(1024, tiles));
    const int c = std::max(512, ceil_div(Kp, want));
    return ceil_div(c, BK2) * BK2;
}

size_t gemm_cn_bf16_part_bytes(int M, int N, int K, int chunk_hint) {
    const int Kp = bf16_ld(K);
    const int ns = std::max(1, ceil_div(Kp, cn_bf16_chunk(M, N, Kp, chunk_hint)));
    return (size_t)ns * M * N * sizeof(c32) + 256;
}

int proj_dapply_bf16(int M, int N, int K, const void *Bpk, int64_t ldb, const void *psi_pk, int64_t ldp,
                     const double *dmat, const int *blo, const int *bn, const int *bdoff, void *Q, void *part,
                     int chunk_hint, hipStream_t st) {
    if (M <= 0 || N <= 0) return ABACUS_PW_OK;
    const int Kp = bf16_ld(K);
    const int c = cn_bf16_chunk(M, N, Kp, chunk_hint);
    const int ns = std::max(1, ceil_div(Kp, c));
    dim3 grid(ceil_div(M, T2), ceil_div(N, T2), ns);
    {
        KernelTimer kt("gemm_cn_bf16", st);
        hipLaunchKernelGGL((k_bf16_t128<true, false>), grid, dim3(256), 0, st, M, N, Kp, c,
                           static_cast<const uint32_t *>(Bpk), ldb, static_cast<const uint32_t *>(psi_pk), ldp, part,
                           (int64_t)0, 0);
        APW_TRY(check_launch("gemm_cn_bf16"));
    }
    return reduce_dapply_f32(M, N, ns, part, dmat, blo, bn, bdoff, Q, st);
}

// Bound over every M' <= M, N' <= N: a chunk is never below 512 k, so at most ceil(Kp / 512) splits.
size_t gemm_cn_bf16_of_f64_bytes(int M, int N, int K) {
    const int Kp = bf16_ld(K);
    const size_t packs = sizeof(uint32_t) * (size_t)(M + N) * Kp;
    return (packs + 255) / 256 * 256 + (size_t)ceil_div(Kp, 512) * M * N * sizeof(c32) + 256;
}

int gemm_cn_bf16_of_f64(int M, int N, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
                        int64_t ldc, void *scratch, hipStream_t st) {
    if (M <= 0 || N <= 0) return ABACUS_PW_OK;
    const int Kp = bf16_ld(K);
    uint32_t *apk = static_cast<uint32_t *>(scratch);
    uint32_t *bpk = apk + (size_t)M * Kp;
    void *part = static_cast<char *>(scratch) + (sizeof(uint32_t) * (size_t)(M + N) * Kp + 255) / 256 * 256;
    APW_TRY(pack_bf16_rows(M, K, A, 1, lda, apk, Kp, st));
    APW_TRY(pack_bf16_rows(N, K, B, 1, ldb, bpk, Kp, st));
    const int c = cn_bf16_chunk(M, N, Kp, 0);
    const int ns = std::max(1, ceil_div(Kp, c));
    dim3 grid(ceil_div(M, T2), ceil_div(N, T2), ns);
    {
        KernelTimer kt("gemm_cn_bf16", st);
        hipLaunchKernelGGL((k_bf16_t128<true, false>), grid, dim3(256), 0, st, M, N, Kp, c, apk, (int64_t)Kp, bpk,
                           (int64_t)Kp, part, (int64_t)0, 0);
        APW_TRY(check_launch("gemm_cn_bf16"));
    }
    return reduce_parts_f32_to_f64(M, N, ns, part, C, ldc, 1.0, 0.0, st);
}

int gemm_nn_bf16_into_f64(int N, int G, int K, const void *Apk, int64_t lda, const void *BTpk, int64_t ldbt, void *C,
                          int64_t ldc, hipStream_t st) {
    if (N <= 0 || G <= 0) return ABACUS_PW_OK;
    const int Kp = bf16_ld(K);
    // band tiles fastest: the blocks that read one tile of the transposed beta run together, so
    // beta streams from HBM once while the small Q is re-read from cache
    dim3 grid(ceil_div(N, T2), ceil_div(G, T2), 1);
    KernelTimer kt("gemm_nn_bf16", st);
    hipLaunchKernelGGL((k_bf16_t128<false, true>), grid, dim3(256), 0, st, G, N, Kp, Kp,
                       static_cast<const uint32_t *>(BTpk), ldbt, static_cast<const uint32_t *>(Apk), lda, C, ldc, 1);
    return check_launch("gemm_nn_bf16");
}

}  // namespace apw

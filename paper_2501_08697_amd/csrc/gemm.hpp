// Complex GEMMs on MFMA; see gemm.hip. prec: 0 complex128, 1 complex64.
#pragma once

#include "common.hpp"

namespace apw {

// Bytes of split-K partial sums gemm_cn / proj_dapply need.
size_t gemm_cn_part_bytes(int M, int N, int K, int elem_bytes, int chunk_hint);

// C[j*ldc + i] = alpha * sum_k conj(A[i*lda + k]) B[j*ldb + k] + beta * C[...],  i < M, j < N.
int gemm_cn(int prec, int M, int N, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
            int64_t ldc, double alpha, double beta, void *part, int chunk_hint, hipStream_t st);

// P[j][i] = <beta_i | psi_j> (M = nproj, N = bands, K = npw); Q[j][i] = sum_t D_blk(i) P[j][.].
// P may be NULL. D-block tables as in the plan.
int proj_dapply(int prec, int M, int N, int K, const void *Bm, int64_t ldb, const void *psi, int64_t ldp,
                const double *dmat, const int *blo, const int *bn, const int *bdoff, void *P, void *Q, void *part,
                int chunk_hint, hipStream_t st);

// C[j*ldc + g] = alpha * sum_i A[j*lda + i] B[i*ldb + g] + beta * C[...],  j < M, g < G.
// gemm_cn on complex128 A, B, C with FP32 products: the operands are rounded to
// complex64 as they are staged, partial sums are FP32, the split-K sum and C are FP64
// (the subspace projection of the reduced-precision Davidson phase).
int gemm_cn_f32_of_f64(int M, int N, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
                       int64_t ldc, double alpha, double beta, void *part, int chunk_hint, hipStream_t st);

int gemm_nn(int prec, int M, int G, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
            int64_t ldc, double alpha, double beta, hipStream_t st);

// As gemm_nn on complex128 A, B and C with FP32 products: the operands are rounded to
// complex64 as they are staged, C accumulates in FP64 (basis updates of the
// reduced-precision Davidson phase).
int gemm_nn_f32_of_f64(int M, int G, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
                       int64_t ldc, double alpha, double beta, hipStream_t st);

// As gemm_nn with complex64 A and B accumulated into a complex128 C.
int gemm_nn_f32_into_f64(int M, int G, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
                         int64_t ldc, double alpha, double beta, hipStream_t st);

// grad_d entry (i, lo+t) of each atom block (+)= sum_n Re(Q[n][i] conj(P[n][lo+t])); P, Q are [nb][M].
int grad_d_accumulate(int prec, int nb, int M, const void *P, const void *Q, const int *blo, const int *bn,
                      const int *bdoff, double *gd, int first, hipStream_t st);

// Split-K sum of complex64 partials [nsplit][N][M] followed by the D blocks: Q[j][i] (complex64).
int reduce_dapply_f32(int M, int N, int nsplit, const void *part, const double *dmat, const int *blo, const int *bn,
                      const int *bdoff, void *Q, hipStream_t st);

// ---- BF16 operands, FP32 accumulation (gemm_bf16.hip) ----
// Leading dimension of packed bf16 rows of K values: K rounded up to a multiple of 32.
inline int bf16_ld(int K) { return (K + 31) / 32 * 32; }
// out[r][c] = in[r][c] (complex128 when in_is_f64, else complex64) rounded to a packed bf16 pair
// (re low, im high) for c < K, 0 for K <= c < ldo.
int pack_bf16_rows(int rows, int K, const void *in, int in_is_f64, int64_t ldi, void *out, int64_t ldo,
                   hipStream_t st);
size_t gemm_cn_bf16_part_bytes(int M, int N, int K, int chunk_hint);
// Q[j][i] = sum_t D_blk(i) P[j][.], P[j][i] = <beta_i|psi_j> with bf16 operands: Bpk packed bf16 beta
// [M][ldb], psi_pk packed bf16 psi [N][ldp], both with zero-padded rows (ldb, ldp = bf16_ld(K)).
int proj_dapply_bf16(int M, int N, int K, const void *Bpk, int64_t ldb, const void *psi_pk, int64_t ldp,
                     const double *dmat, const int *blo, const int *bn, const int *bdoff, void *Q, void *part,
                     int chunk_hint, hipStream_t st);
// C = alpha sum_s part[s] + beta C: complex64 split-K partials [nsplit][N][M] into complex128 C (ldc).
int reduce_parts_f32_to_f64(int M, int N, int nsplit, const void *part, void *C, int64_t ldc, double alpha,
                            double beta, hipStream_t st);
// C = A^H B (M x N, ldc) for complex128 rows A [M][lda], B [N][ldb] of length K, computed with both
// operands rounded to bf16 and FP32 accumulation; scratch of gemm_cn_bf16_of_f64_bytes(M, N, K) bytes.
size_t gemm_cn_bf16_of_f64_bytes(int M, int N, int K);
int gemm_cn_bf16_of_f64(int M, int N, int K, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
                        int64_t ldc, void *scratch, hipStream_t st);
// out[g][i] = in[i][g] (complex128 [rows][ldi], g < cols) as packed bf16, zero for rows <= i < ldo.
int pack_bf16_transpose(int rows, int cols, const void *in, int64_t ldi, void *out, int64_t ldo, hipStream_t st);
// C[j][g] += sum_i A[j][i] B[i][g] for j < N, g < G, i < K: Apk packed bf16 A [N][lda], BTpk packed bf16
// transposed B [G][ldbt], lda and ldbt = bf16_ld(K) with zero padding; C complex128 [N][ldc].
int gemm_nn_bf16_into_f64(int N, int G, int K, const void *Apk, int64_t lda, const void *BTpk, int64_t ldbt, void *C,
                          int64_t ldc, hipStream_t st);

}  // namespace apw

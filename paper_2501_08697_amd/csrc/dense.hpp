// Small dense FP64 linear algebra on the GPU; see dense.hip.
#pragma once

#include "common.hpp"

namespace apw {

constexpr int kSmallSub = 1024;  // largest order of the one-CU kernels (their LDS arrays)
constexpr int kMaxSub = 4096;    // largest eigen-problem order handled on the device
constexpr int kMaxChol = 1024;   // largest Cholesky order (the explicit inverse holds a column in registers)
constexpr int kLargeHeevMin = 257;   // orders from here on take the multi-CU eigensolver (dense_large.hip)
constexpr int kLargeCholMin = 137;   // orders from here on take the blocked multi-CU Cholesky

// G (n x n, row-major, ld) Hermitian positive definite: lower triangle := L with
// G = L L^H; Linv (ldi) := L^{-1}. *info_dev = 0 or k + 1 for a failed pivot.
// scratch: potrf_scratch_bytes(n) bytes of device memory (unused for small n).
int potrf_inv(int n, z64 *G, int ld, z64 *Linv, int ldi, int *info_dev, void *scratch, hipStream_t st);
size_t potrf_scratch_bytes(int n);

size_t heev_scratch_bytes(int n);

// Lowest nw eigenpairs of the Hermitian A (n x n, row-major, ld; destroyed):
// w[0..nw) ascending; coef[j*ldc + i] = i-th component of the j-th eigenvector.
int heev_lowest(int n, z64 *A, int ld, int nw, double *w, z64 *coef, int ldc, void *scratch, hipStream_t st);

}  // namespace apw

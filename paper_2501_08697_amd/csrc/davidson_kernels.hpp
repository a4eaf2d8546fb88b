// Per-band and small-matrix kernels of the block Davidson iteration; see davidson_kernels.hip.
#pragma once

#include "common.hpp"

namespace apw {

int dav_resid(int nb, int npw, const z64 *X, const z64 *W, const double *lam, const double *kin, z64 *R, double *rn2,
              double *ek, hipStream_t st);
int dav_precond(int m, int npw, const int *act, const z64 *R, const double *kin, const double *ek, z64 *T,
                hipStream_t st);
int dav_row_norm2(int m, int npw, const z64 *T, double *out, hipStream_t st);
int dav_gather_rows(int m, int npw, const int *idx, const z64 *src, z64 *dst, hipStream_t st);
int dav_hs_append(int nb0, int m, const z64 *C, int ldc, z64 *Hs, int ld, hipStream_t st);
int dav_hs_diag(int n, const double *theta, z64 *Hs, int ld, hipStream_t st);
int dav_copy_block(int n, const z64 *src, int lds, z64 *dst, int ldd, hipStream_t st);
int dav_lowdin(int n, z64 *G, hipStream_t st);
int dav_add_diag(int n, z64 *G, int ld, double s, hipStream_t st);

}  // namespace apw

// Local-potential term of H psi (grid transforms); see local.hip.
#pragma once

#include <functional>

#include "plan.hpp"

namespace apw {

// 1 when a transform of length n is compiled in.
int local_length_supported(int n);
// OK when the plan's grid can run at fft_prec (0 = FP64, 1 = FP32), else EBAD_FFT_SIZE.
int local_supported(const Plan &P, int fft_prec);
// Slab work space for nbands bands.
size_t local_slab_bytes(const Plan &P, int fft_prec, int nbands);

// hpsi = |k+G|^2 psi + (V psi) for nb bands at the k-points [k0, k1): psi and hpsi start at
// k0's [nb][npw_k] block, k blocks back to back. Each band batch runs every k-point in one
// launch per pass. fft_prec: 0 FP64, 1 FP32 transforms. io_prec: 0 complex128, 1 complex64.
// vloc: float64 grid for fft_prec 0, float32 for 1. slab: local_slab_bytes((k1-k0) band_batch).
// after_batch(b0, bbt), if given, is called once the kernels of bands [b0, b0+bbt)
// are enqueued (their H psi rows are complete when that work has run on st).
int local_term(const Plan &P, int k0, int k1, int fft_prec, int io_prec, const void *vloc, const void *psi,
               void *hpsi, int nb, void *slab, int band_batch, hipStream_t st,
               const std::function<int(int, int)> &after_batch = nullptr);

// Inverse y-z transforms of bands [b0, b0+bbt) at the k-points [k0, k1) into slab planes
// (virtual band (k - k0) * bbt + b); psi starts at k0's block of nb bands.
int local_inverse_planes(const Plan &P, int k0, int k1, int nb, int b0, int bbt, int fft_prec, int io_prec,
                         const void *psi, void *slab, hipStream_t st);
// part[g] (+)= sum over bands b = g (mod G) of Re(conj(gamma_b(r)) psi_b(r)), from the slab planes of
// psi (slab_x) and dY (slab_y); part is [G][N1][N2][N3]; first != 0 overwrites.
int local_gradv_accumulate(const Plan &P, int fft_prec, const void *slab_x, const void *slab_y, int nbands,
                           double *part, int G, int first, hipStream_t st);
// part[g] (+)= sum over bands b = g (mod G) of w_b |psi_b(r)|^2 from the slab planes of psi;
// virtual band b = kk * bbt + j of the batch has w_b = occ[kk * nb + b0 + j].
int local_density_accumulate(const Plan &P, int fft_prec, const void *slab, int nbands, const double *occ, int nb,
                             int b0, int bbt, double *part, int G, int first, hipStream_t st);
// out = scale * sum_g part[g]   (fixed order)
int local_sum_parts(const Plan &P, const double *part, int G, double scale, double *out, hipStream_t st);

}  // namespace apw

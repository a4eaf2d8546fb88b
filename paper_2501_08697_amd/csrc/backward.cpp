// Adjoint of H psi (abacus_pw_apply_h_backward). For a real loss L with
// upstream dY = dL/d(H psi) in PyTorch's complex convention:
//   grad_psi = H dY                                  (H is Hermitian)
//   grad_V(r_j) = (1/N) sum_{k,n} Re(conj(gamma_n(r_j)) psi_n(r_j)),
//       gamma_n and psi_n the unnormalised inverse grid transforms of dY_n, psi_n
//   grad_D[a](i,j) = Re sum_{k,n} Q_in conj(P_jn),  P = B^H psi, Q = B^H dY
// The grids are recomputed from psi and dY (nothing is kept from a forward
// call). Band and k sums run in a fixed order, so results repeat bit for bit.
// The band density shares the grid-gradient machinery (one transform per band).
#include <algorithm>

#include "gemm.hpp"
#include "hamiltonian.hpp"
#include "local.hpp"

namespace apw {

constexpr int kGradVGroups = 8;

int apply_h_backward_all(const abacus_pw_problem &p, Plan &P, int prec, int nb, const void *psi, const void *dy,
                         void *grad_psi, double *grad_v, double *grad_d, hipStream_t st) {
    const int fp = prec == ABACUS_PW_FP64 ? 0 : 1;   // transforms and GEMMs
    const int io = prec == ABACUS_PW_FP32 ? 1 : 0;
    const size_t ib = io == 0 ? 16 : 8;
    APW_TRY(local_supported(P, fp));
    if (grad_psi) APW_TRY(apply_h_all(p, P, prec, nb, dy, grad_psi, st));
    if (grad_d && P.nproj > 0) {
        APW_TRY(operator_copies(p, P, false, fp == 1, st));
        APW_TRY(P.proj.ensure((size_t)nb * P.nproj * ib));
        APW_TRY(P.proj2.ensure((size_t)nb * P.nproj * ib));
        APW_TRY(P.gemm_part.ensure(gemm_cn_part_bytes(P.nproj, nb, P.max_npw, (int)ib, g_splitk_chunk)));
        for (int k = 0; k < P.nk; ++k) {
            const KTables &K = P.k[k];
            const void *bk = fp == 0 ? static_cast<const void *>(static_cast<const char *>(p.beta) + (size_t)P.nproj * K.pw_off * 16)
                                     : static_cast<const void *>(P.beta32.as<char>() + (size_t)P.nproj * K.pw_off * 8);
            const char *xk = static_cast<const char *>(psi) + (size_t)nb * K.pw_off * ib;
            const char *yk = static_cast<const char *>(dy) + (size_t)nb * K.pw_off * ib;
            APW_TRY(gemm_cn(fp, P.nproj, nb, K.npw, bk, K.npw, xk, K.npw, P.proj.ptr, P.nproj, 1.0, 0.0,
                            P.gemm_part.ptr, g_splitk_chunk, st));
            APW_TRY(gemm_cn(fp, P.nproj, nb, K.npw, bk, K.npw, yk, K.npw, P.proj2.ptr, P.nproj, 1.0, 0.0,
                            P.gemm_part.ptr, g_splitk_chunk, st));
            APW_TRY(grad_d_accumulate(fp, nb, P.nproj, P.proj.ptr, P.proj2.ptr, P.proj_blk_lo, P.proj_blk_n,
                                      P.proj_blk_doff, grad_d, k == 0, st));
        }
    }
    if (grad_v) {
        const int bb = default_band_batch(P, nb);
        const size_t sb = local_slab_bytes(P, fp, P.nk * bb);
        APW_TRY(P.slab.ensure(sb));
        APW_TRY(P.slab2.ensure(sb));
        APW_TRY(P.gradv_part.ensure(sizeof(double) * (size_t)kGradVGroups * P.N));
        int first = 1;
        for (int b0 = 0; b0 < nb; b0 += bb) {
            const int n = std::min(bb, nb - b0);
            APW_TRY(local_inverse_planes(P, 0, P.nk, nb, b0, n, fp, io, psi, P.slab.ptr, st));
            APW_TRY(local_inverse_planes(P, 0, P.nk, nb, b0, n, fp, io, dy, P.slab2.ptr, st));
            APW_TRY(local_gradv_accumulate(P, fp, P.slab.ptr, P.slab2.ptr, P.nk * n, P.gradv_part.as<double>(),
                                           kGradVGroups, first, st));
            first = 0;
        }
        APW_TRY(local_sum_parts(P, P.gradv_part.as<double>(), kGradVGroups, 1.0 / (double)P.N, grad_v, st));
    }
    return ABACUS_PW_OK;
}

// Band density (abacus_pw_density): rho(r_j) = sum_{k,n} occ[k][n] |psi_nk(r_j)|^2, psi_nk(r)
// the unnormalised inverse transform of the coefficients. Per band batch the y-z
// inverse transforms of every k-point write slab planes, then one x pass
// transforms them and adds the weighted squared moduli; the G partial grids are
// summed in a fixed order at the end.
int density_all(const abacus_pw_problem &p, Plan &P, int prec, int nb, const void *psi, const double *occ,
                double *rho, hipStream_t st) {
    (void)p;
    const int fp = prec == ABACUS_PW_FP64 ? 0 : 1;
    const int io = prec == ABACUS_PW_FP32 ? 1 : 0;
    APW_TRY(local_supported(P, fp));
    const int bb = default_band_batch(P, nb);
    APW_TRY(P.slab.ensure(local_slab_bytes(P, fp, P.nk * bb)));
    APW_TRY(P.gradv_part.ensure(sizeof(double) * (size_t)kGradVGroups * P.N));
    int first = 1;
    for (int b0 = 0; b0 < nb; b0 += bb) {
        const int n = std::min(bb, nb - b0);
        APW_TRY(local_inverse_planes(P, 0, P.nk, nb, b0, n, fp, io, psi, P.slab.ptr, st));
        APW_TRY(local_density_accumulate(P, fp, P.slab.ptr, P.nk * n, occ, nb, b0, n, P.gradv_part.as<double>(),
                                         kGradVGroups, first, st));
        first = 0;
    }
    return local_sum_parts(P, P.gradv_part.as<double>(), kGradVGroups, 1.0, rho, st);
}

}  // namespace apw

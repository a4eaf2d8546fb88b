// H psi over every k-point: the local term on the grid (local.hip) followed
// by the Kleinman-Bylander term as two MFMA GEMMs (gemm.hip):
//   P = B^H psi  (nproj x nb per k),  Q = D P (atom blocks),  H psi += B Q.
#include "hamiltonian.hpp"

#include <algorithm>

#include "convert.hpp"
#include "gemm.hpp"
#include "local.hpp"

namespace apw {

int default_band_batch(const Plan &P, int nb) {
    int bb = g_band_batch > 0 ? g_band_batch : 64;
    (void)P;
    return std::max(1, std::min(bb, nb));
}

// Reduced-precision copies of V and beta, refreshed unless the caller marks the operator static.
int operator_copies(const abacus_pw_problem &p, Plan &P, bool need_v32, bool need_b32, hipStream_t st, bool need_bf) {
    const bool stat = (p.flags & ABACUS_PW_STATIC_OPERATOR) != 0;
    if (need_v32 && !(stat && P.vloc32_src == p.vloc)) {
        APW_TRY(P.vloc32.ensure(sizeof(float) * (size_t)P.N));
        APW_TRY(convert_f64_to_f32(P.N, p.vloc, P.vloc32.as<float>(), st));
        P.vloc32_src = p.vloc;
    }
    if (need_b32 && P.nproj > 0 && !(stat && P.beta32_src == p.beta)) {
        const int64_t n = 2 * (int64_t)P.nproj * P.npw_total;
        APW_TRY(P.beta32.ensure(sizeof(float) * (size_t)n));
        APW_TRY(convert_f64_to_f32(n, static_cast<const double *>(p.beta), P.beta32.as<float>(), st));
        P.beta32_src = p.beta;
    }
    if (need_bf && P.nproj > 0 && !(stat && P.betabf_src == p.beta)) {
        const int64_t n = (int64_t)P.nproj * P.npw_total;
        APW_TRY(P.betabf.ensure(sizeof(uint32_t) * (size_t)n));
        APW_TRY(pack_bf16(n, p.beta, P.betabf.ptr, st));
        P.betabf_src = p.beta;
    }
    return ABACUS_PW_OK;
}

// H psi for nb bands of k-point k: psi, hpsi are that k's [nb][npw_k] blocks.
// H psi for nb bands at the k-points [k0, k1): psi and hpsi start at k0's [nb][npw_k] block.
// The local term runs every k-point of a band batch in one launch per pass; the
// projector GEMMs run per k-point.
int apply_h_range(const abacus_pw_problem &p, Plan &P, int k0, int k1, int prec, int nb, const void *psi, void *hpsi,
                  hipStream_t st, bool refresh_copies) {
    const bool bf = prec == ABACUS_PW_MIXED_BF16;
    const int fft_prec = prec == ABACUS_PW_FP64 ? 0 : 1;
    const int io_prec = prec == ABACUS_PW_FP32 ? 1 : 0;
    const int gemm_prec = prec == ABACUS_PW_FP64 ? 0 : 1;
    const size_t ib = io_prec == 0 ? 16 : 8;     // bytes per psi element
    APW_TRY(local_supported(P, fft_prec));
    const int bb = default_band_batch(P, nb);
    APW_TRY(P.slab.ensure(local_slab_bytes(P, fft_prec, (k1 - k0) * bb)));
    if (refresh_copies) APW_TRY(operator_copies(p, P, fft_prec == 1, gemm_prec == 1 && !bf, st, bf));
    const void *v = fft_prec == 0 ? static_cast<const void *>(p.vloc) : P.vloc32.ptr;
    APW_TRY(local_term(P, k0, k1, fft_prec, io_prec, v, psi, hpsi, nb, P.slab.ptr, bb, st));
    if (P.nproj == 0) return ABACUS_PW_OK;
    const size_t gb = gemm_prec == 0 ? 16 : 8;   // bytes per GEMM operand element
    APW_TRY(P.projq.ensure((size_t)nb * P.nproj * gb));
    if (bf)
        APW_TRY(P.gemm_part.ensure(gemm_cn_bf16_part_bytes(P.nproj, nb, P.max_npw, g_splitk_chunk)));
    else
        APW_TRY(P.gemm_part.ensure(gemm_cn_part_bytes(P.nproj, nb, P.max_npw, (int)gb, g_splitk_chunk)));
    if (prec == ABACUS_PW_MIXED_FP32) APW_TRY(P.tmp_io.ensure((size_t)nb * P.max_npw * 8));
    for (int k = k0; k < k1; ++k) {
        const KTables &K = P.k[k];
        const size_t eoff = (size_t)nb * (K.pw_off - P.pw_off[k0]);
        const char *xk = static_cast<const char *>(psi) + eoff * ib;
        char *yk = static_cast<char *>(hpsi) + eoff * ib;
        if (bf) {
            const void *bk = P.betabf.as<char>() + (size_t)P.nproj * K.pw_off * 4;
            APW_TRY(proj_dapply_bf16(P.nproj, nb, K.npw, bk, K.npw, xk, 1, K.npw, p.dmat, P.proj_blk_lo, P.proj_blk_n,
                                     P.proj_blk_doff, P.projq.ptr, P.gemm_part.ptr, g_splitk_chunk, st));
            APW_TRY(gemm_nn_bf16_into_f64(nb, K.npw, P.nproj, P.projq.ptr, P.nproj, bk, K.npw, yk, K.npw, st));
            continue;
        }
        const void *bk = gemm_prec == 0
                             ? static_cast<const void *>(static_cast<const char *>(p.beta) + (size_t)P.nproj * K.pw_off * 16)
                             : static_cast<const void *>(P.beta32.as<char>() + (size_t)P.nproj * K.pw_off * 8);
        const void *xg = xk;
        if (prec == ABACUS_PW_MIXED_FP32) {
            APW_TRY(convert_f64_to_f32(2 * (int64_t)nb * K.npw, reinterpret_cast<const double *>(xk),
                                       P.tmp_io.as<float>(), st));
            xg = P.tmp_io.ptr;
        }
        APW_TRY(proj_dapply(gemm_prec, P.nproj, nb, K.npw, bk, K.npw, xg, K.npw, p.dmat, P.proj_blk_lo, P.proj_blk_n,
                            P.proj_blk_doff, nullptr, P.projq.ptr, P.gemm_part.ptr, g_splitk_chunk, st));
        if (prec == ABACUS_PW_MIXED_FP32)
            APW_TRY(gemm_nn_f32_into_f64(nb, K.npw, P.nproj, P.projq.ptr, P.nproj, bk, K.npw, yk, K.npw, 1.0, 1.0, st));
        else
            APW_TRY(gemm_nn(gemm_prec, nb, K.npw, P.nproj, P.projq.ptr, P.nproj, bk, K.npw, yk, K.npw, 1.0, 1.0, st));
    }
    return ABACUS_PW_OK;
}

int apply_h_k(const abacus_pw_problem &p, Plan &P, int k, int prec, int nb, const void *psi, void *hpsi,
              hipStream_t st, bool refresh_copies) {
    return apply_h_range(p, P, k, k + 1, prec, nb, psi, hpsi, st, refresh_copies);
}

int apply_h_all(const abacus_pw_problem &p, Plan &P, int prec, int nb, const void *psi, void *hpsi, hipStream_t st) {
    return apply_h_range(p, P, 0, P.nk, prec, nb, psi, hpsi, st, true);
}

}  // namespace apw

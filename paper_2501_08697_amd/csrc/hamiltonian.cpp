// H psi over every k-point: the local term on the grid (local.hip) and the
// Kleinman-Bylander term as two MFMA GEMMs (gemm.hip):
//   P = B^H psi  (nproj x nb per k),  Q = D P (atom blocks),  H psi += B Q.
#include "hamiltonian.hpp"

#include <algorithm>
#include <mutex>

#include "convert.hpp"
#include "gemm.hpp"
#include "local.hpp"

namespace apw {

int default_band_batch(const Plan &P, int nb) {
    int bb = g_band_batch > 0 ? g_band_batch : 64;
    (void)P;
    return std::max(1, std::min(bb, nb));
}

// Start (in packed words per projector row) of k-point k's block of the padded bf16 beta copy.
int64_t bf16_offset(const Plan &P, int k) {
    int64_t o = 0;
    for (int q = 0; q < k; ++q) o += bf16_ld(P.npw[q]);
    return o;
}

// Allocates the plan's reduced-precision operator copies without filling them.
int operator_copy_buffers(Plan &P, bool need_v32, bool need_b32, bool need_bf) {
    if (need_v32) APW_TRY(P.vloc32.ensure(sizeof(float) * (size_t)P.N));
    if (need_b32 && P.nproj > 0) APW_TRY(P.beta32.ensure(sizeof(float) * 2 * (size_t)P.nproj * P.npw_total));
    if (need_bf && P.nproj > 0) {
        APW_TRY(P.betabf.ensure(sizeof(uint32_t) * (size_t)P.nproj * (size_t)bf16_offset(P, P.nk)));
        APW_TRY(P.betabfT.ensure(sizeof(uint32_t) * (size_t)bf16_ld(P.nproj) * (size_t)P.npw_total));
    }
    return ABACUS_PW_OK;
}

// Reduced-precision copies of V and beta, refreshed unless the caller marks the operator static.
// A conversion recorded into a stream capture has not run when the call returns (it runs at
// each replay), so it does not mark the copy as made: the next eager call converts again.
int operator_copies(const abacus_pw_problem &p, Plan &P, bool need_v32, bool need_b32, hipStream_t st, bool need_bf) {
    const bool stat = (p.flags & ABACUS_PW_STATIC_OPERATOR) != 0;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    APW_HIP(hipStreamIsCapturing(st, &cap));
    const bool capturing = cap != hipStreamCaptureStatusNone;
    APW_TRY(operator_copy_buffers(P, need_v32, need_b32, need_bf));
    if (need_v32 && !(stat && P.vloc32_src == p.vloc)) {
        APW_TRY(convert_f64_to_f32(P.N, p.vloc, P.vloc32.as<float>(), st));
        P.vloc32_src = capturing ? nullptr : p.vloc;
    }
    if (need_b32 && P.nproj > 0 && !(stat && P.beta32_src == p.beta)) {
        const int64_t n = 2 * (int64_t)P.nproj * P.npw_total;
        APW_TRY(convert_f64_to_f32(n, static_cast<const double *>(p.beta), P.beta32.as<float>(), st));
        P.beta32_src = capturing ? nullptr : p.beta;
    }
    if (need_bf && P.nproj > 0 && !(stat && P.betabf_src == p.beta)) {
        // per k a [nproj][bf16_ld(npw_k)] block of packed bf16 pairs, rows zero-padded
        for (int k = 0; k < P.nk; ++k) {
            const int npw = P.npw[k];
            APW_TRY(pack_bf16_rows(P.nproj, npw, static_cast<const z64 *>(p.beta) + (size_t)P.nproj * P.pw_off[k], 1,
                                   npw, P.betabf.as<uint32_t>() + (size_t)P.nproj * bf16_offset(P, k), bf16_ld(npw),
                                   st));
        }
        // and per k the transposed [npw_k][bf16_ld(nproj)] block, projector index contiguous
        const int ldq = bf16_ld(P.nproj);
        for (int k = 0; k < P.nk; ++k)
            APW_TRY(pack_bf16_transpose(P.nproj, P.npw[k], static_cast<const z64 *>(p.beta) + (size_t)P.nproj * P.pw_off[k],
                                        P.npw[k], P.betabfT.as<uint32_t>() + (size_t)ldq * P.pw_off[k], ldq, st));
        P.betabf_src = capturing ? nullptr : p.beta;
    }
    return ABACUS_PW_OK;
}

namespace {

// A second stream per device (default priority, non-blocking) on which the
// projector GEMMs run beside the local term. Events fork it from the caller's
// stream and join it back before the call returns.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, step = nullptr, join = nullptr;
};
constexpr int kMaxDevices = 64;
std::mutex g_side_mu;
SideStream g_side[kMaxDevices];

int side_stream(SideStream **out) {
    int dev = 0;
    APW_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(ABACUS_PW_EINTERNAL, "device index out of range");
    std::lock_guard<std::mutex> l(g_side_mu);
    SideStream &ss = g_side[dev];
    if (!ss.s) {
        APW_HIP(hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking));
        APW_HIP(hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming));
        APW_HIP(hipEventCreateWithFlags(&ss.step, hipEventDisableTiming));
        APW_HIP(hipEventCreateWithFlags(&ss.join, hipEventDisableTiming));
    }
    *out = &ss;
    return ABACUS_PW_OK;
}

// Work enqueued on `to` after this call runs after the work already on `from`.
int order(hipEvent_t e, hipStream_t from, hipStream_t to) {
    APW_HIP(hipEventRecord(e, from));
    APW_HIP(hipStreamWaitEvent(to, e, 0));
    return ABACUS_PW_OK;
}

}  // namespace

// H psi for nb bands at the k-points [k0, k1): psi and hpsi start at k0's [nb][npw_k] block.
// The local term runs every k-point of a band batch in one launch per pass and
// writes hpsi = (T + V) psi; the projector GEMMs run per k-point: the
// projections Q_k = D B_k^H psi_k, then hpsi += B_k Q_k. With the overlap knob on
// the projections start on the side stream at once and each band batch's B Q
// follows there as soon as that batch's local term is done, so the GEMMs share
// the GPU with the plane passes. Off by default: on the 72^3 / 23847-PW case the
// concurrent kernels slow each other down about as much as they overlap.
// Bytes of the per-call work buffers of apply_h_range for nb bands at [k0, k1) (current knobs).
void hwork_sizes(const Plan &P, int prec, int nb, int k0, int k1, size_t sz[kHWorkParts]) {
    const bool bf = prec == ABACUS_PW_MIXED_BF16;
    const int fft_prec = prec == ABACUS_PW_FP64 ? 0 : 1;
    const int gemm_prec = prec == ABACUS_PW_FP64 ? 0 : 1;
    for (int i = 0; i < kHWorkParts; ++i) sz[i] = 0;
    sz[0] = local_slab_bytes(P, fft_prec, (k1 - k0) * default_band_batch(P, nb));
    if (P.nproj == 0) return;
    const size_t gb = gemm_prec == 0 ? 16 : 8;
    sz[1] = (size_t)nb * P.nproj * gb * (k1 - k0);
    if (bf) {
        for (int k = k0; k < k1; ++k) sz[2] = std::max(sz[2], gemm_cn_bf16_part_bytes(P.nproj, nb, P.npw[k], g_splitk_chunk));
        sz[3] = sizeof(uint32_t) * (size_t)nb * bf16_ld(P.max_npw);
        sz[4] = sizeof(uint32_t) * (size_t)nb * bf16_ld(P.nproj);
    } else {
        sz[2] = gemm_cn_part_bytes(P.nproj, nb, P.max_npw, (int)gb, g_splitk_chunk);
    }
    if (prec == ABACUS_PW_MIXED_FP32) sz[5] = (size_t)nb * P.max_npw * 8;
}

size_t hwork_total(const size_t sz[kHWorkParts]) {
    size_t t = 0;
    for (int i = 0; i < kHWorkParts; ++i) t += (sz[i] + 255) / 256 * 256;
    return t;
}

int apply_h_range(const abacus_pw_problem &p, Plan &P, int k0, int k1, int prec, int nb, const void *psi, void *hpsi,
                  hipStream_t st, bool refresh_copies, void *ext_ws, size_t ext_bytes) {
    const bool bf = prec == ABACUS_PW_MIXED_BF16;
    const int fft_prec = prec == ABACUS_PW_FP64 ? 0 : 1;
    const int io_prec = prec == ABACUS_PW_FP32 ? 1 : 0;
    const int gemm_prec = prec == ABACUS_PW_FP64 ? 0 : 1;
    const size_t ib = io_prec == 0 ? 16 : 8;     // bytes per psi element
    APW_TRY(local_supported(P, fft_prec));
    const int bb = default_band_batch(P, nb);
    // work buffers: the plan's (grown as needed) or carved from the caller's work space
    size_t sz[kHWorkParts];
    hwork_sizes(P, prec, nb, k0, k1, sz);
    void *w[kHWorkParts] = {};
    if (ext_ws) {
        if (ext_bytes < hwork_total(sz))
            return set_error(ABACUS_PW_EBAD_SHAPE, "work space smaller than abacus_pw_workspace_size");
        char *c = static_cast<char *>(ext_ws);
        for (int i = 0; i < kHWorkParts; ++i) {
            w[i] = sz[i] ? c : nullptr;
            c += (sz[i] + 255) / 256 * 256;
        }
    } else {
        DeviceBuffer *bufs[kHWorkParts] = {&P.slab, &P.projq, &P.gemm_part, &P.psibf, &P.qbf, &P.tmp_io};
        for (int i = 0; i < kHWorkParts; ++i)
            if (sz[i]) {
                APW_TRY(bufs[i]->ensure(sz[i]));
                w[i] = bufs[i]->ptr;
            }
    }
    void *slab = w[0], *projq = w[1], *gemm_part = w[2], *psibf = w[3], *qbf = w[4], *tmp_io = w[5];
    if (refresh_copies) APW_TRY(operator_copies(p, P, fft_prec == 1, gemm_prec == 1 && !bf, st, bf));
    const void *v = fft_prec == 0 ? static_cast<const void *>(p.vloc) : P.vloc32.ptr;
    if (P.nproj == 0) return local_term(P, k0, k1, fft_prec, io_prec, v, psi, hpsi, nb, slab, bb, st);

    const size_t gb = gemm_prec == 0 ? 16 : 8;   // bytes per element of Q (complex64 in the BF16 mode)
    const size_t qk = (size_t)nb * P.nproj * gb; // Q bytes per k-point

    const bool overlap = g_overlap == 1;
    SideStream *ss = nullptr;
    hipStream_t gs = st;
    if (overlap) {
        APW_TRY(side_stream(&ss));
        gs = ss->s;
        APW_TRY(order(ss->fork, st, gs));
    }
    auto beta_k = [&](const KTables &K) -> const void * {
        if (bf) return P.betabf.as<char>() + (size_t)P.nproj * bf16_offset(P, (int)(&K - P.k.data())) * 4;
        return gemm_prec == 0 ? static_cast<const void *>(static_cast<const char *>(p.beta) + (size_t)P.nproj * K.pw_off * 16)
                              : static_cast<const void *>(P.beta32.as<char>() + (size_t)P.nproj * K.pw_off * 8);
    };
    // Q_k = D B_k^H psi_k
    for (int k = k0; k < k1; ++k) {
        const KTables &K = P.k[k];
        const char *xk = static_cast<const char *>(psi) + (size_t)nb * (K.pw_off - P.pw_off[k0]) * ib;
        void *qk_ptr = static_cast<char *>(projq) + qk * (k - k0);
        const void *bk = beta_k(K);
        if (bf) {
            const int ldk = bf16_ld(K.npw);
            APW_TRY(pack_bf16_rows(nb, K.npw, xk, io_prec == 0 ? 1 : 0, K.npw, psibf, ldk, gs));
            APW_TRY(proj_dapply_bf16(P.nproj, nb, K.npw, bk, ldk, psibf, ldk, p.dmat, P.proj_blk_lo,
                                     P.proj_blk_n, P.proj_blk_doff, qk_ptr, gemm_part, g_splitk_chunk, gs));
            continue;
        }
        const void *xg = xk;
        if (prec == ABACUS_PW_MIXED_FP32) {
            APW_TRY(convert_f64_to_f32(2 * (int64_t)nb * K.npw, reinterpret_cast<const double *>(xk),
                                       static_cast<float *>(tmp_io), gs));
            xg = tmp_io;
        }
        APW_TRY(proj_dapply(gemm_prec, P.nproj, nb, K.npw, bk, K.npw, xg, K.npw, p.dmat, P.proj_blk_lo, P.proj_blk_n,
                            P.proj_blk_doff, nullptr, qk_ptr, gemm_part, g_splitk_chunk, gs));
    }
    // hpsi[b0 .. b0+bbt) += B_k Q_k[b0 .. b0+bbt) for every k-point
    auto add_bq = [&](int b0, int bbt, hipStream_t s) -> int {
        for (int k = k0; k < k1; ++k) {
            const KTables &K = P.k[k];
            char *yk = static_cast<char *>(hpsi) + ((size_t)nb * (K.pw_off - P.pw_off[k0]) + (size_t)b0 * K.npw) * ib;
            const char *qb = static_cast<char *>(projq) + qk * (k - k0) + (size_t)b0 * P.nproj * gb;
            const void *bk = beta_k(K);
            if (bf) {
                const int ldq = bf16_ld(P.nproj);
                APW_TRY(pack_bf16_rows(bbt, P.nproj, qb, 0, P.nproj, qbf, ldq, s));
                const uint32_t *btk = P.betabfT.as<uint32_t>() + (size_t)ldq * K.pw_off;
                APW_TRY(gemm_nn_bf16_into_f64(bbt, K.npw, P.nproj, qbf, ldq, btk, ldq, yk, K.npw, s));
            }
            else if (prec == ABACUS_PW_MIXED_FP32)
                APW_TRY(gemm_nn_f32_into_f64(bbt, K.npw, P.nproj, qb, P.nproj, bk, K.npw, yk, K.npw, 1.0, 1.0, s));
            else
                APW_TRY(gemm_nn(gemm_prec, bbt, K.npw, P.nproj, qb, P.nproj, bk, K.npw, yk, K.npw, 1.0, 1.0, s));
        }
        return ABACUS_PW_OK;
    };
    if (!overlap) {
        APW_TRY(local_term(P, k0, k1, fft_prec, io_prec, v, psi, hpsi, nb, slab, bb, st));
        return add_bq(0, nb, st);
    }
    APW_TRY(local_term(P, k0, k1, fft_prec, io_prec, v, psi, hpsi, nb, slab, bb, st, [&](int b0, int bbt) -> int {
        APW_TRY(order(ss->step, st, gs));
        return add_bq(b0, bbt, gs);
    }));
    return order(ss->join, gs, st);
}

int apply_h_k(const abacus_pw_problem &p, Plan &P, int k, int prec, int nb, const void *psi, void *hpsi,
              hipStream_t st, bool refresh_copies) {
    return apply_h_range(p, P, k, k + 1, prec, nb, psi, hpsi, st, refresh_copies);
}

int apply_h_all(const abacus_pw_problem &p, Plan &P, int prec, int nb, const void *psi, void *hpsi, hipStream_t st,
                void *ws, size_t ws_bytes) {
    return apply_h_range(p, P, 0, P.nk, prec, nb, psi, hpsi, st, true, ws, ws_bytes);
}

int apply_h_workspace(Plan &P, int prec, int nb, size_t *bytes) {
    const bool bf = prec == ABACUS_PW_MIXED_BF16;
    const int fft_prec = prec == ABACUS_PW_FP64 ? 0 : 1;
    const int gemm_prec = prec == ABACUS_PW_FP64 ? 0 : 1;
    APW_TRY(local_supported(P, fft_prec));
    APW_TRY(operator_copy_buffers(P, fft_prec == 1, gemm_prec == 1 && !bf, bf));
    if (g_overlap == 1) {
        SideStream *ss = nullptr;
        APW_TRY(side_stream(&ss));
    }
    size_t sz[kHWorkParts];
    hwork_sizes(P, prec, nb, 0, P.nk, sz);
    *bytes = hwork_total(sz);
    return ABACUS_PW_OK;
}

}  // namespace apw

// Band-by-band preconditioned conjugate-gradient eigensolver (abacus_pw_cg),
// the CG figure of Sec. III.B. For band i at k-point k:
//
//  1. psi_i -= sum_{j<i} psi_j <psi_j|psi_i>; normalise; p = H psi_i;
//     lambda = <psi_i|p>.
//  2. Repeat until ||p - lambda psi_i|| < tol or max_iter steps:
//       r = p - lambda psi_i; g = K r (Teter-Payne-Allan, from the band's kinetic
//       energy); g -= sum_{j<=i} psi_j <psi_j|g>;
//       gamma = max(0, Re<g|r - r_prev> / Re<g_prev|r_prev>) (Polak-Ribiere, 0 at
//       the first step); d = g + gamma d; d_hat = (d - psi_i <psi_i|d>) / norm;
//       h = H d_hat; theta = atan2(-2 Re<p|d_hat>, <d_hat|h> - lambda) / 2;
//       psi_i = cos(theta) psi_i + sin(theta) d_hat; p likewise with h;
//       lambda = <psi_i|p>.
//
// H acts on one band at a time (the band-by-band order of the method is
// sequential). The scalars of a step (inner products, gamma, theta) stay in
// device memory (cg_kernels.hip): the host reads them once per step, for the
// convergence test. Projections against the lower bands use the MFMA GEMMs.
#include <cmath>
#include <vector>

#include "cg_kernels.hpp"
#include "davidson_kernels.hpp"
#include "gemm.hpp"
#include "hamiltonian.hpp"
#include "local.hpp"

namespace apw {

namespace {

struct CgBuffers {
    DeviceBuffer p, r0, r1, g, d, dh, h, coef, part, scal, act;
};

// x -= X[0..m) X[0..m)^H x  (rows of X are orthonormal bands)
int project_out(int m, int npw, const z64 *X, z64 *x, CgBuffers &b, hipStream_t st) {
    if (m <= 0) return ABACUS_PW_OK;
    APW_TRY(gemm_cn(0, m, 1, npw, X, npw, x, npw, b.coef.ptr, m, 1.0, 0.0, b.part.ptr, 0, st));
    return gemm_nn(0, 1, npw, m, b.coef.ptr, m, X, npw, x, npw, -1.0, 1.0, st);
}

int cg_k(const abacus_pw_problem &p, Plan &P, int k, int nb, z64 *X, CgBuffers &b, double tol, int max_iter,
         double *eig, double *resid, int *iters, bool &converged, hipStream_t st) {
    const int npw = P.k[k].npw;
    const double *kin = P.k[k].kin;
    const size_t vb = sizeof(z64) * (size_t)npw;
    APW_TRY(b.p.ensure(vb));
    APW_TRY(b.r0.ensure(vb));
    APW_TRY(b.r1.ensure(vb));
    APW_TRY(b.g.ensure(vb));
    APW_TRY(b.d.ensure(vb));
    APW_TRY(b.dh.ensure(vb));
    APW_TRY(b.h.ensure(vb));
    APW_TRY(b.coef.ensure(sizeof(z64) * (size_t)nb));
    APW_TRY(b.part.ensure(gemm_cn_part_bytes(nb, 1, npw, 16, 0)));
    APW_TRY(b.scal.ensure(sizeof(CgScalars)));
    APW_TRY(b.act.ensure(sizeof(int)));
    const int zero = 0;
    APW_HIP(hipMemcpyAsync(b.act.ptr, &zero, sizeof(int), hipMemcpyHostToDevice, st));
    CgScalars *S = b.scal.as<CgScalars>();
    z64 *pv = b.p.as<z64>(), *g = b.g.as<z64>(), *d = b.d.as<z64>(), *dh = b.dh.as<z64>(), *h = b.h.as<z64>();
    z64 *r = b.r0.as<z64>(), *rprev = b.r1.as<z64>();
    CgScalars hs;
    for (int i = 0; i < nb; ++i) {
        z64 *x = X + (size_t)i * npw;
        APW_TRY(project_out(i, npw, X, x, b, st));
        APW_TRY(cg_dots(npw, x, x, &S->rn2, nullptr, nullptr, nullptr, true, st));
        APW_TRY(cg_stage_scale_self(S, st));
        APW_TRY(cg_axpby(npw, &S->a1, x, &S->b1, x, x, st));
        APW_TRY(apply_h_k(p, P, k, ABACUS_PW_FP64, 1, x, pv, st, false));
        APW_TRY(cg_dots(npw, x, pv, &S->lam, nullptr, nullptr, nullptr, true, st));
        APW_TRY(cg_zero(npw, d, st));
        int step = 0;
        for (;;) {
            // r = p - lambda psi, ||r||^2, E_kin(psi)
            APW_TRY(dav_resid(1, npw, x, pv, &S->lam, kin, r, &S->rn2, &S->ek, st));
            APW_HIP(hipMemcpyAsync(&hs, S, sizeof(CgScalars), hipMemcpyDeviceToHost, st));
            APW_HIP(hipStreamSynchronize(st));
            if (!(std::sqrt(hs.rn2) >= tol) || step >= max_iter) break;
            // g = K r with bands 0..i projected out
            APW_TRY(dav_precond(1, npw, b.act.as<int>(), r, kin, &S->ek, g, st));
            APW_TRY(project_out(i + 1, npw, X, g, b, st));
            // Polak-Ribiere direction
            APW_TRY(cg_dots(npw, g, r, &S->gr, step > 0 ? g : nullptr, rprev, &S->grp, true, st));
            APW_TRY(cg_stage_direction(S, step == 0 ? 1 : 0, st));
            APW_TRY(cg_axpby(npw, &S->a1, g, &S->b1, d, d, st));
            // step direction: d without its psi component, normalised
            APW_TRY(cg_dots(npw, x, d, &S->xd.re, nullptr, nullptr, nullptr, false, st));
            APW_TRY(cg_stage_project(S, st));
            APW_TRY(cg_axpby(npw, &S->a1, d, &S->b1, x, dh, st));
            APW_TRY(cg_dots(npw, dh, dh, &S->dn2, nullptr, nullptr, nullptr, true, st));
            APW_TRY(cg_stage_normalise(S, st));
            APW_TRY(cg_axpby(npw, &S->a1, dh, &S->b1, dh, dh, st));
            // exact line minimisation on span{psi, d_hat}
            APW_TRY(apply_h_k(p, P, k, ABACUS_PW_FP64, 1, dh, h, st, false));
            APW_TRY(cg_dots(npw, pv, dh, &S->b, dh, h, &S->c, true, st));
            APW_TRY(cg_stage_rotate(S, st));
            APW_TRY(cg_axpby(npw, &S->a1, x, &S->b1, dh, x, st));
            APW_TRY(cg_axpby(npw, &S->a1, pv, &S->b1, h, pv, st));
            APW_TRY(cg_dots(npw, x, pv, &S->lam, nullptr, nullptr, nullptr, true, st));
            std::swap(r, rprev);
            ++step;
        }
        eig[i] = hs.lam;
        resid[i] = std::sqrt(hs.rn2);
        iters[i] = step;
        converged = converged && std::sqrt(hs.rn2) < tol;
    }
    return ABACUS_PW_OK;
}

}  // namespace

int cg_all(const abacus_pw_problem &p, Plan &P, int nb, void *psi, double *eig, double tol, int max_iter, int *iters,
           double *resid, hipStream_t st) {
    APW_TRY(local_supported(P, 0));
    CgBuffers b;
    bool converged = true;
    std::vector<double> e(nb), rn(nb);
    std::vector<int> it(nb);
    for (int k = 0; k < P.nk; ++k) {
        z64 *X = static_cast<z64 *>(psi) + (size_t)nb * P.k[k].pw_off;
        APW_TRY(cg_k(p, P, k, nb, X, b, tol, max_iter, e.data(), rn.data(), it.data(), converged, st));
        for (int n = 0; n < nb; ++n) {
            eig[(size_t)k * nb + n] = e[n];
            if (resid) resid[(size_t)k * nb + n] = rn[n];
            if (iters) iters[(size_t)k * nb + n] = it[n];
        }
    }
    APW_HIP(hipStreamSynchronize(st));
    return converged ? ABACUS_PW_OK : ABACUS_PW_NOT_CONVERGED;
}

}  // namespace apw

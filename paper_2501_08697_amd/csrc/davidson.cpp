// Block Davidson driver (abacus_pw_davidson). Sec. III.B names Davidson as
// the plane-wave eigensolver without listing its steps; the steps here are:
//
//  1. Cholesky-QR of the initial block X; W = H X; Rayleigh-Ritz on span(X).
//  2. Repeat: residuals R = W - X Lambda and their FP64 norms; stop when every
//     norm < tol. Teter-Payne-Allan preconditioned corrections for the
//     unconverged bands. When the basis would exceed ndim * nb vectors it
//     restarts from the current Ritz vectors and locks the bands that have
//     converged (their pairs leave the Rayleigh-Ritz problem). Two classical
//     Gram-Schmidt passes against the locked vectors and the basis,
//     corrections whose norm fell below 1e-10 of their pre-projection norm are
//     dropped, Cholesky-QR twice; append T and H T to the basis; Rayleigh-Ritz
//     on the whole basis keeping the lowest nb - (locked) pairs.
//
// Every vector operation runs on the device: GEMMs on MFMA, Cholesky and the
// Hermitian eigensolver in FP64 (dense.hip). The host only reads the residual
// norms (and the Cholesky status) once per iteration to steer the loop.
//
// Mixed modes: a first Davidson phase applies H in reduced precision (FP32
// transforms, FP32 or BF16 projector GEMMs, complex128 vectors) and forms the
// subspace matrix V^H H V with FP32 (MIXED_FP32) or bf16 (MIXED_BF16) products
// on MFMA with FP32 accumulation and an FP64 split-K sum;
// orthonormalisation, Cholesky, Rayleigh-Ritz and residual norms stay FP64.
// Then an FP64 phase refines the Ritz vectors to tol with the FP64 H.
#include <algorithm>
#include <cmath>
#include <vector>

#include "davidson_kernels.hpp"
#include "dense.hpp"
#include "gemm.hpp"
#include "hamiltonian.hpp"
#include "local.hpp"

namespace apw {

namespace {

struct Buffers {
    DeviceBuffer V, HV, Xc, Wc, R, Y, Hs, Hw, coef, C, G, Linv, part, theta, rn2, ek, n0, n1, act, idx, info, heev, bfs,
        chol, info2;
};

// Pinned host staging for the index lists uploaded each iteration: the copies are
// enqueued without waiting, and a list is rewritten only after the next read-back
// (which waits for the stream) has ordered it behind its copy.
struct HostLists {
    int *act = nullptr, *keep = nullptr, *idx = nullptr;
    double *theta = nullptr;
    int n = 0;
    ~HostLists() {
        if (theta) (void)hipHostFree(theta);
    }
    int ensure(int m) {
        if (m <= n) return ABACUS_PW_OK;
        if (theta) APW_HIP(hipHostFree(theta));
        void *p = nullptr;
        APW_HIP(hipHostMalloc(&p, (sizeof(double) + sizeof(int) * 3) * (size_t)m, hipHostMallocDefault));
        theta = static_cast<double *>(p);   // the doubles first, so every array is aligned
        act = reinterpret_cast<int *>(theta + m);
        keep = act + m;
        idx = keep + m;
        n = m;
        return ABACUS_PW_OK;
    }
};

// The dense subspace steps under their own profile names ("eigensolver:", "cholesky:"),
// so that the "subspace:" records hold only the counted products.
int potrf_inv_s(int n, z64 *G, int ld, z64 *Li, int ldi, int *info, void *scratch, hipStream_t st) {
    ProfScope ps("cholesky");
    return potrf_inv(n, G, ld, Li, ldi, info, scratch, st);
}

// Flops of a subspace product (complex, 8 M N K) for the per-kernel profile.
void sub_flops(const char *label, double M, double N, double K) { prof_count_flops(label, 8.0 * M * N * K); }

// Enqueue an upload from pinned host memory (no wait).
int h2d_async(void *dst, const void *src, size_t bytes, hipStream_t st) {
    APW_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    return ABACUS_PW_OK;
}

int d2h(void *dst, const void *src, size_t bytes, hipStream_t st) {
    APW_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
    APW_HIP(hipStreamSynchronize(st));
    return ABACUS_PW_OK;
}

int h2d(void *dst, const void *src, size_t bytes, hipStream_t st) {
    APW_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    APW_HIP(hipStreamSynchronize(st));   // the host array may change right after
    return ABACUS_PW_OK;
}

int d2d(void *dst, const void *src, size_t bytes, hipStream_t st) {
    APW_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
    return ABACUS_PW_OK;
}

// One Cholesky-QR pass without a wait: Y = L^{-1} T with G = T^H T = L L^H; the
// pivot status goes to *info_dev (the caller reads it later). T is unchanged.
int cholqr_pass_async(int m, int npw, const z64 *T, z64 *Y, Buffers &b, int *info_dev, hipStream_t st) {
    z64 *G = b.G.as<z64>(), *Linv = b.Linv.as<z64>();
    APW_TRY(gemm_cn(0, m, m, npw, T, npw, T, npw, G, m, 1.0, 0.0, b.part.ptr, 0, st));
    sub_flops("gemm_cn", m, m, npw);
    APW_TRY(potrf_inv_s(m, G, m, Linv, m, info_dev, b.chol.ptr, st));
    sub_flops("gemm_nn", m, npw, m);
    return gemm_nn(0, m, npw, m, Linv, m, T, npw, Y, npw, 1.0, 0.0, st);
}

// Orthonormalise the m rows of T (length npw) by `passes` Cholesky-QR passes;
// Y is scratch of the same size. A Gram matrix that is not numerically
// positive definite is retried once with the shift of shifted Cholesky-QR.
int cholqr_rows(int m, int npw, z64 *T, z64 *Y, Buffers &b, int passes, hipStream_t st) {
    z64 *G = b.G.as<z64>(), *Linv = b.Linv.as<z64>();
    for (int pass = 0; pass < passes; ++pass) {
        APW_TRY(gemm_cn(0, m, m, npw, T, npw, T, npw, G, m, 1.0, 0.0, b.part.ptr, 0, st));
        sub_flops("gemm_cn", m, m, npw);
        APW_TRY(potrf_inv_s(m, G, m, Linv, m, b.info.as<int>(), b.chol.ptr, st));
        int info = 0;
        APW_TRY(d2h(&info, b.info.ptr, sizeof(int), st));
        if (info != 0) {
            std::vector<double> nrm(m);
            APW_TRY(dav_row_norm2(m, npw, T, b.n1.as<double>(), st));
            APW_TRY(d2h(nrm.data(), b.n1.ptr, sizeof(double) * m, st));
            double tr = 0.0;
            for (double x : nrm) tr += x;
            const double shift = 11.0 * ((double)m * npw + (double)m * (m + 1)) * 2.220446049250313e-16 * tr;
            APW_TRY(gemm_cn(0, m, m, npw, T, npw, T, npw, G, m, 1.0, 0.0, b.part.ptr, 0, st));
            sub_flops("gemm_cn", m, m, npw);
            APW_TRY(dav_add_diag(m, G, m, shift, st));
            APW_TRY(potrf_inv_s(m, G, m, Linv, m, b.info.as<int>(), b.chol.ptr, st));
            APW_TRY(d2h(&info, b.info.ptr, sizeof(int), st));
            if (info != 0) return set_error(ABACUS_PW_ECHOLESKY, "Gram matrix is not positive definite");
            ++passes;   // a shifted pass is followed by one more plain pass
            if (passes > 4) passes = 4;
        }
        APW_TRY(gemm_nn(0, m, npw, m, Linv, m, T, npw, Y, npw, 1.0, 0.0, st));
        sub_flops("gemm_nn", m, npw, m);
        APW_TRY(d2d(T, Y, sizeof(z64) * (size_t)m * npw, st));
    }
    return ABACUS_PW_OK;
}

// Rayleigh-Ritz on the n x n subspace matrix in Hw: lowest nb eigenpairs, then one
// first-order Lowdin step M = 1.5 I - 0.5 C C^H on the coefficient rows, which
// turns the inverse-iteration vectors (orthonormal to ~eps ||T|| / gap) into an
// orthonormal set to O(1e-17). Returns the coefficient rows (ld nmax) in *out.
int rayleigh_ritz(int n, int nb, int nmax, Buffers &b, z64 **out, hipStream_t st) {
    z64 *Hw = b.Hw.as<z64>(), *coef = b.coef.as<z64>(), *G = b.G.as<z64>();
    {
        ProfScope ps("eigensolver");
        APW_TRY(heev_lowest(n, Hw, nmax, nb, b.theta.as<double>(), coef, nmax, b.heev.ptr, st));
    }
    APW_TRY(gemm_cn(0, nb, nb, n, coef, nmax, coef, nmax, G, nb, 1.0, 0.0, b.part.ptr, 0, st));
    sub_flops("gemm_cn", nb, nb, n);
    APW_TRY(dav_lowdin(nb, G, st));
    APW_TRY(gemm_nn(0, nb, n, nb, G, nb, coef, nmax, Hw, nmax, 1.0, 0.0, st));
    sub_flops("gemm_nn", nb, n, nb);
    *out = Hw;
    return ABACUS_PW_OK;
}

struct Result {
    int iters = 0;
    bool converged = false;
};

// One Davidson phase at k-point k on the [nb][npw] block X (in/out).
// hprec: precision of H. stagnation > 0 stops the phase early when the largest
// residual has not dropped below 0.7 of its best value for that many iterations.
//
// Locking: at each restart, bands whose residual is below tol leave the
// Rayleigh-Ritz problem. Their vectors stay fixed as the first nl rows of V,
// corrections are orthogonalised against them together with the basis that
// follows them in V, and Rayleigh-Ritz keeps the lowest nA = nb - nl pairs.
// The output merges both sets in ascending order of their Ritz values.
int davidson_k(const abacus_pw_problem &p, Plan &P, int k, int hprec, int nb, z64 *X, Buffers &b, HostLists &hl,
               double tol, int max_iter, int ndim, int stagnation, std::vector<double> &theta_h,
               std::vector<double> &rn_h, Result &res, hipStream_t st) {
    ProfScope prof_scope("subspace");   // per-kernel profile: this solver's own kernels
    const int npw = P.k[k].npw, nmax = ndim * nb;
    const double *kin = P.k[k].kin;
    if (nmax > kMaxSub) return set_error(ABACUS_PW_EBAD_SHAPE, "ndim * nb exceeds the device eigensolver limit (4096)");
    if (nb > kMaxChol) return set_error(ABACUS_PW_EBAD_SHAPE, "nb exceeds the device Cholesky limit (1024)");
    const size_t vb = sizeof(z64) * (size_t)npw;
    const int vrows = nmax + nb;   // locked rows (at most nb - 1), then the basis
    APW_TRY(b.V.ensure(vb * vrows));
    APW_TRY(b.HV.ensure(vb * nmax));
    APW_TRY(b.Xc.ensure(vb * nb));
    APW_TRY(b.Wc.ensure(vb * nb));
    APW_TRY(b.R.ensure(vb * nb));
    APW_TRY(b.Y.ensure(vb * nb));
    APW_TRY(b.Hs.ensure(sizeof(z64) * (size_t)nmax * nmax));
    APW_TRY(b.Hw.ensure(sizeof(z64) * (size_t)nmax * nmax));
    APW_TRY(b.coef.ensure(sizeof(z64) * (size_t)nb * nmax));
    APW_TRY(b.C.ensure(sizeof(z64) * (size_t)vrows * nb));
    APW_TRY(b.G.ensure(sizeof(z64) * (size_t)nb * nb));
    APW_TRY(b.Linv.ensure(sizeof(z64) * (size_t)nb * nb));
    APW_TRY(b.part.ensure(std::max(gemm_cn_part_bytes(vrows, nb, npw, 16, 0), gemm_cn_part_bytes(nb, nb, npw, 16, 0))));
    APW_TRY(b.theta.ensure(sizeof(double) * nmax));
    APW_TRY(b.rn2.ensure(sizeof(double) * nb));
    APW_TRY(b.ek.ensure(sizeof(double) * nb));
    APW_TRY(b.n0.ensure(sizeof(double) * 2 * nb + 64));   // norms before, then after the projection
    APW_TRY(b.n1.ensure(sizeof(double) * nb));
    APW_TRY(b.act.ensure(sizeof(int) * nb));
    APW_TRY(b.idx.ensure(sizeof(int) * nb));
    APW_TRY(b.info.ensure(sizeof(int)));
    APW_TRY(b.info2.ensure(sizeof(int)));
    APW_TRY(hl.ensure(nb));
    APW_TRY(b.heev.ensure(heev_scratch_bytes(nmax)));
    APW_TRY(b.chol.ensure(potrf_scratch_bytes(nb)));
    z64 *V = b.V.as<z64>(), *HV = b.HV.as<z64>(), *Xc = b.Xc.as<z64>(), *Wc = b.Wc.as<z64>(), *R = b.R.as<z64>();
    z64 *Y = b.Y.as<z64>(), *Hs = b.Hs.as<z64>(), *Hw = b.Hw.as<z64>(), *C = b.C.as<z64>();
    double *theta = b.theta.as<double>();

    // 1. Cholesky-QR, H X, Rayleigh-Ritz on span(X)
    APW_TRY(d2d(Xc, X, vb * nb, st));
    APW_TRY(cholqr_rows(nb, npw, Xc, Y, b, 1, st));
    {
        ProfScope hs(nullptr);   // H psi keeps the plain kernel names
        APW_TRY(apply_h_k(p, P, k, hprec, nb, Xc, Wc, st, false));
    }
    // subspace projections V^H (H V): FP32 products in a reduced-precision phase, else FP64
    // subspace projections V^H (H V): FP64, or in the reduced-precision phase FP32 (MIXED_FP32) or
    // bf16 (MIXED_BF16) products with FP32 accumulation
    if (hprec == ABACUS_PW_MIXED_BF16) APW_TRY(b.bfs.ensure(gemm_cn_bf16_of_f64_bytes(nmax, nb, npw)));
    auto project = [&](int M, int N, const z64 *A, const z64 *B, z64 *Cout, int ldc) -> int {
        sub_flops(hprec == ABACUS_PW_MIXED_BF16 ? "gemm_cn_bf16" : "gemm_cn", M, N, npw);
        if (hprec == ABACUS_PW_FP64) return gemm_cn(0, M, N, npw, A, npw, B, npw, Cout, ldc, 1.0, 0.0, b.part.ptr, 0, st);
        if (hprec == ABACUS_PW_MIXED_BF16)
            return gemm_cn_bf16_of_f64(M, N, npw, A, npw, B, npw, Cout, ldc, b.bfs.ptr, st);
        return gemm_cn_f32_of_f64(M, N, npw, A, npw, B, npw, Cout, ldc, 1.0, 0.0, b.part.ptr, 0, st);
    };
    // basis products of the iteration (the projection against the basis, the basis
    // updates to the Ritz vectors): FP64, or in the bf16 phase (which stops at a residual
    // of 1e-3) FP32 products on the FP64 vectors with FP64 results. The FP32 phase, which
    // goes to 1e-5, keeps them FP64: with FP32 products there its iterations to 1e-8 at
    // 72^3 rose from 39 to 68. Cholesky-QR and the residuals stay FP64.
    const bool low = hprec == ABACUS_PW_MIXED_BF16;
    auto basis_cn = [&](int M, int N, const z64 *A, const z64 *B, z64 *Cout, int ldc) -> int {
        sub_flops("gemm_cn", M, N, npw);
        return low ? gemm_cn_f32_of_f64(M, N, npw, A, npw, B, npw, Cout, ldc, 1.0, 0.0, b.part.ptr, 0, st)
                   : gemm_cn(0, M, N, npw, A, npw, B, npw, Cout, ldc, 1.0, 0.0, b.part.ptr, 0, st);
    };
    auto basis_nn = [&](int M, int K, const z64 *A, int lda, const z64 *B, z64 *Cout, double alpha,
                        double beta) -> int {
        sub_flops("gemm_nn", M, npw, K);
        return low ? gemm_nn_f32_of_f64(M, npw, K, A, lda, B, npw, Cout, npw, alpha, beta, st)
                   : gemm_nn(0, M, npw, K, A, lda, B, npw, Cout, npw, alpha, beta, st);
    };
    APW_TRY(project(nb, nb, Xc, Wc, C, nb));
    APW_TRY(dav_hs_append(0, nb, C, nb, Hs, nmax, st));
    APW_TRY(dav_copy_block(nb, Hs, nmax, Hw, nmax, st));
    z64 *rc = nullptr;
    APW_TRY(rayleigh_ritz(nb, nb, nmax, b, &rc, st));
    APW_TRY(gemm_nn(0, nb, npw, nb, rc, nmax, Xc, npw, V, npw, 1.0, 0.0, st));
    APW_TRY(gemm_nn(0, nb, npw, nb, rc, nmax, Wc, npw, HV, npw, 1.0, 0.0, st));
    sub_flops("gemm_nn", 2.0 * nb, npw, nb);
    APW_TRY(d2d(Xc, V, vb * nb, st));
    APW_TRY(d2d(Wc, HV, vb * nb, st));
    APW_TRY(dav_hs_diag(nb, theta, Hs, nmax, st));
    int nbasis = nb;   // basis rows, stored after the nl locked rows of V
    int nA = nb, nl = 0;
    std::vector<double> thL, rnL, thA(nb);

    std::vector<double> rn2(nb), n0(nb), n1(nb);
    std::vector<int> act, conv, keep;
    double best = INFINITY;
    int since_best = 0;
    res = Result{};
    double *nrm0 = b.n0.as<double>(), *nrm1 = nrm0 + nb;   // correction norms before / after the projection
    bool check_info2 = false;   // the last iteration's second Cholesky-QR pass has a status to read
    // Host crossings per iteration: one read of the residual norms (with the status of the
    // previous second Cholesky-QR pass), one read of the correction norms with the status of
    // the first pass, which runs before that read on every correction; uploads of index lists
    // are enqueued from pinned memory without a wait.
    for (;;) {
        z64 *Vb = V + (size_t)nl * npw;
        APW_TRY(dav_resid(nA, npw, Xc, Wc, theta, kin, R, b.rn2.as<double>(), b.ek.as<double>(), st));
        int info2 = 0;
        APW_HIP(hipMemcpyAsync(rn2.data(), b.rn2.ptr, sizeof(double) * nA, hipMemcpyDeviceToHost, st));
        if (check_info2) APW_HIP(hipMemcpyAsync(&info2, b.info2.ptr, sizeof(int), hipMemcpyDeviceToHost, st));
        APW_HIP(hipStreamSynchronize(st));
        if (info2 != 0)
            return set_error(ABACUS_PW_ECHOLESKY, "second Cholesky-QR pass of the corrections not positive definite");
        act.clear();
        conv.clear();
        double worst = 0.0;
        for (int n = 0; n < nA; ++n) {
            const double r = std::sqrt(rn2[n]);
            worst = std::max(worst, r);
            (r < tol ? conv : act).push_back(n);
        }
        if (act.empty()) {
            res.converged = true;
            break;
        }
        if (res.iters >= max_iter) break;
        if (stagnation > 0) {
            if (worst < 0.7 * best) {
                best = worst;
                since_best = 0;
            } else if (++since_best >= stagnation) {
                break;
            }
        }
        int m = (int)act.size();
        std::copy(act.begin(), act.end(), hl.act);
        APW_TRY(h2d_async(b.act.ptr, hl.act, sizeof(int) * m, st));
        const bool restart = nbasis + m > nmax;
        z64 *T;
        if (restart && !conv.empty()) {
            // lock the converged bands: their vectors join the locked rows, the
            // active ones become the new basis
            const int nc = (int)conv.size();
            APW_TRY(dav_precond(m, npw, b.act.as<int>(), R, kin, b.ek.as<double>(), Y, st));
            std::copy(conv.begin(), conv.end(), hl.idx);
            APW_TRY(h2d_async(b.idx.ptr, hl.idx, sizeof(int) * nc, st));
            APW_TRY(dav_gather_rows(nc, npw, b.idx.as<int>(), Xc, Vb, st));
            Vb = V + (size_t)(nl + nc) * npw;
            APW_TRY(dav_gather_rows(m, npw, b.act.as<int>(), Xc, Vb, st));
            APW_TRY(dav_gather_rows(m, npw, b.act.as<int>(), Wc, HV, st));
            APW_TRY(d2d(Xc, Vb, vb * m, st));
            APW_TRY(d2d(Wc, HV, vb * m, st));
            APW_TRY(d2h(thA.data(), theta, sizeof(double) * nA, st));
            for (int i : conv) {
                thL.push_back(thA[i]);
                rnL.push_back(std::sqrt(rn2[i]));
            }
            for (int i = 0; i < m; ++i) hl.theta[i] = thA[act[i]];
            APW_TRY(h2d_async(theta, hl.theta, sizeof(double) * m, st));
            nl += nc;
            nA = m;
            nbasis = m;
            APW_TRY(dav_hs_diag(nA, theta, Hs, nmax, st));
            T = Vb + (size_t)nbasis * npw;
            APW_TRY(d2d(T, Y, vb * m, st));
        } else {
            if (restart) {
                APW_TRY(d2d(Vb, Xc, vb * nA, st));
                APW_TRY(d2d(HV, Wc, vb * nA, st));
                APW_TRY(dav_hs_diag(nA, theta, Hs, nmax, st));
                nbasis = nA;
            }
            T = Vb + (size_t)nbasis * npw;
            APW_TRY(dav_precond(m, npw, b.act.as<int>(), R, kin, b.ek.as<double>(), T, st));
        }
        z64 *HT = HV + (size_t)nbasis * npw;
        const int north = nl + nbasis;   // locked rows and basis, contiguous in V
        APW_TRY(dav_row_norm2(m, npw, T, nrm0, st));
        for (int pass = 0; pass < 2; ++pass) {
            APW_TRY(basis_cn(north, m, V, T, C, north));
            APW_TRY(basis_nn(m, north, C, north, V, T, -1.0, 1.0));
        }
        APW_TRY(dav_row_norm2(m, npw, T, nrm1, st));
        // first Cholesky-QR pass on every correction (Y = L^{-1} T), before the drop test
        // is known: it is kept when nothing is dropped and its pivots are positive
        APW_TRY(cholqr_pass_async(m, npw, T, Y, b, b.info.as<int>(), st));
        int info1 = 0;
        APW_HIP(hipMemcpyAsync(n0.data(), nrm0, sizeof(double) * m, hipMemcpyDeviceToHost, st));
        APW_HIP(hipMemcpyAsync(n1.data(), nrm1, sizeof(double) * m, hipMemcpyDeviceToHost, st));
        APW_HIP(hipMemcpyAsync(&info1, b.info.ptr, sizeof(int), hipMemcpyDeviceToHost, st));
        APW_HIP(hipStreamSynchronize(st));
        keep.clear();
        for (int i = 0; i < m; ++i)
            if (std::sqrt(n1[i]) >= 1e-10 * std::sqrt(n0[i])) keep.push_back(i);
        check_info2 = false;
        if ((int)keep.size() < m) {
            // corrections fell into the basis: drop them, then Cholesky-QR on the rest
            if (!keep.empty()) {
                std::copy(keep.begin(), keep.end(), hl.keep);
                APW_TRY(h2d_async(b.act.ptr, hl.keep, sizeof(int) * keep.size(), st));
                APW_TRY(dav_gather_rows((int)keep.size(), npw, b.act.as<int>(), T, Y, st));
                APW_TRY(d2d(T, Y, vb * keep.size(), st));
            }
            m = (int)keep.size();
            if (m == 0) break;
            APW_TRY(cholqr_rows(m, npw, T, Y, b, 2, st));
        } else if (info1 != 0) {
            // not positive definite: Cholesky-QR with the shifted retry
            APW_TRY(cholqr_rows(m, npw, T, Y, b, 2, st));
        } else {
            APW_TRY(d2d(T, Y, vb * m, st));
            APW_TRY(cholqr_pass_async(m, npw, T, Y, b, b.info2.as<int>(), st));
            APW_TRY(d2d(T, Y, vb * m, st));
            check_info2 = true;
        }
        {
            ProfScope hs(nullptr);
            APW_TRY(apply_h_k(p, P, k, hprec, m, T, HT, st, false));
        }
        const int n = nbasis + m;
        APW_TRY(project(n, m, Vb, HT, C, n));
        APW_TRY(dav_hs_append(nbasis, m, C, n, Hs, nmax, st));
        APW_TRY(dav_copy_block(n, Hs, nmax, Hw, nmax, st));
        APW_TRY(rayleigh_ritz(n, nA, nmax, b, &rc, st));
        APW_TRY(basis_nn(nA, n, rc, nmax, Vb, Xc, 1.0, 0.0));
        APW_TRY(basis_nn(nA, n, rc, nmax, HV, Wc, 1.0, 0.0));
        nbasis = n;
        ++res.iters;
    }
    // Ritz pairs of the active block; with locked bands, merge both sets in
    // ascending order of their Ritz values
    APW_TRY(d2h(thA.data(), theta, sizeof(double) * nA, st));
    theta_h.assign(thL.begin(), thL.end());
    rn_h.assign(rnL.begin(), rnL.end());
    for (int n = 0; n < nA; ++n) {
        theta_h.push_back(thA[n]);
        rn_h.push_back(std::sqrt(rn2[n]));
    }
    if (check_info2) {
        int info2 = 0;
        APW_TRY(d2h(&info2, b.info2.ptr, sizeof(int), st));
        if (info2 != 0)
            return set_error(ABACUS_PW_ECHOLESKY, "second Cholesky-QR pass of the corrections not positive definite");
    }
    if (nl == 0) {
        APW_TRY(d2d(X, Xc, vb * nb, st));
    } else {
        std::vector<int> perm(nb);
        for (int i = 0; i < nb; ++i) perm[i] = i;
        std::stable_sort(perm.begin(), perm.end(), [&](int a, int c) { return theta_h[a] < theta_h[c]; });
        z64 *Vb = V + (size_t)nl * npw;
        APW_TRY(d2d(Vb, Xc, vb * nA, st));
        APW_TRY(h2d(b.idx.ptr, perm.data(), sizeof(int) * nb, st));
        APW_TRY(dav_gather_rows(nb, npw, b.idx.as<int>(), V, X, st));
        std::vector<double> ts(nb), rs(nb);
        for (int i = 0; i < nb; ++i) {
            ts[i] = theta_h[perm[i]];
            rs[i] = rn_h[perm[i]];
        }
        theta_h.swap(ts);
        rn_h.swap(rs);
    }
    return ABACUS_PW_OK;
}

}  // namespace

int davidson_all(const abacus_pw_problem &p, Plan &P, int prec, int nb, void *psi, double *eig, double tol,
                 int max_iter, int ndim, int *iters, double *resid, hipStream_t st) {
    APW_TRY(local_supported(P, 0));   // the refinement phase always runs FP64 transforms
    Buffers b;
    HostLists hl;
    bool all = true;
    std::vector<double> th, rn;
    // operator copies once per solve (the reduced-precision phase reads them)
    APW_TRY(operator_copies(p, P, prec != ABACUS_PW_FP64, prec == ABACUS_PW_MIXED_FP32, st,
                            prec == ABACUS_PW_MIXED_BF16));
    for (int k = 0; k < P.nk; ++k) {
        z64 *X = static_cast<z64 *>(psi) + (size_t)nb * P.k[k].pw_off;
        int total = 0;
        Result r;
        if (prec != ABACUS_PW_FP64) {
            // reduced-precision phase: stop at its noise floor (FP32 ~1e-5, BF16 projectors ~1e-3) or on stagnation
            const double tol_a = std::max(tol, prec == ABACUS_PW_MIXED_BF16 ? 1e-3 : 1e-5);
            APW_TRY(davidson_k(p, P, k, prec, nb, X, b, hl, tol_a, max_iter, ndim, 3, th, rn, r, st));
            total += r.iters;
        }
        APW_TRY(davidson_k(p, P, k, ABACUS_PW_FP64, nb, X, b, hl, tol, std::max(0, max_iter - total), ndim, 0, th, rn, r,
                           st));
        total += r.iters;
        all = all && r.converged;
        for (int n = 0; n < nb; ++n) {
            eig[(size_t)k * nb + n] = th[n];
            if (resid) resid[(size_t)k * nb + n] = rn[n];
        }
        if (iters) iters[k] = total;
    }
    APW_HIP(hipStreamSynchronize(st));
    return all ? ABACUS_PW_OK : ABACUS_PW_NOT_CONVERGED;
}

}  // namespace apw

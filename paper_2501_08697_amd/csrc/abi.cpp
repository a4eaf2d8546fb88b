// C entry points, error messages and per-kernel timing.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "abacus_pw.h"
#include "common.hpp"
#include "dense.hpp"
#include "hamiltonian.hpp"
#include "local.hpp"
#include "plan.hpp"

namespace apw {

// ------------------------------------------------------------------ errors --
static thread_local std::string t_err;

int set_error(int code, const std::string &msg) {
    t_err = msg;
    return code;
}

// ----------------------------------------------------------------- timing --
bool g_prof_on = false;
thread_local const char *t_prof_scope = nullptr;
namespace {
struct Pending {
    std::string name;
    hipEvent_t a, b;
};
struct Total {
    long n = 0;
    double ms = 0.0, flops = 0.0;
};
std::mutex g_prof_mu;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
thread_local std::vector<std::pair<std::string, hipEvent_t>> t_open;
std::map<std::string, Total> g_totals;

std::string scoped(const char *name) {
    return t_prof_scope ? std::string(t_prof_scope) + ":" + name : std::string(name);
}

hipEvent_t take_event() {
    std::lock_guard<std::mutex> l(g_prof_mu);
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}
}  // namespace

void prof_begin(const char *name, hipStream_t s) {
    hipEvent_t e = take_event();
    (void)hipEventRecord(e, s);
    t_open.emplace_back(scoped(name), e);
}

void prof_end(hipStream_t s) {
    if (t_open.empty()) return;
    auto [name, a] = t_open.back();
    t_open.pop_back();
    hipEvent_t b = take_event();
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> l(g_prof_mu);
    g_pending.push_back(Pending{std::move(name), a, b});
}

void prof_count_flops(const char *name, double flops) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> l(g_prof_mu);
    g_totals[scoped(name)].flops += flops;
}

static int prof_collect() {
    std::vector<Pending> todo;
    {
        std::lock_guard<std::mutex> l(g_prof_mu);
        todo.swap(g_pending);
    }
    for (auto &p : todo) {
        APW_HIP(hipEventSynchronize(p.b));
        float ms = 0.f;
        APW_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        std::lock_guard<std::mutex> l(g_prof_mu);
        auto &t = g_totals[p.name];
        t.n += 1;
        t.ms += ms;
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    return ABACUS_PW_OK;
}

int plan_reset_all();

// Work space of the dense entry points, one per device, grown as needed.
namespace {
constexpr int kMaxDevicesDense = 64;
std::mutex g_dense_mu;
DeviceBuffer g_dense_ws[kMaxDevicesDense];
DeviceBuffer g_dense_info[kMaxDevicesDense];

int dense_workspace(size_t bytes, void **ws, int **info) {
    int dev = 0;
    APW_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevicesDense) return set_error(ABACUS_PW_EINTERNAL, "device index out of range");
    std::lock_guard<std::mutex> l(g_dense_mu);
    if (g_dense_ws[dev].bytes < bytes) {
        APW_HIP(hipDeviceSynchronize());   // earlier calls may still use the old buffer
        APW_TRY(g_dense_ws[dev].ensure(bytes));
    }
    APW_TRY(g_dense_info[dev].ensure(sizeof(int)));
    *ws = g_dense_ws[dev].ptr;
    *info = g_dense_info[dev].as<int>();
    return ABACUS_PW_OK;
}
}  // namespace

}  // namespace apw

using namespace apw;

template <typename F> static int guarded(F &&f) {
    try {
        return f();
    } catch (const std::exception &e) {
        return set_error(ABACUS_PW_EINTERNAL, std::string("internal error: ") + e.what());
    } catch (...) {
        return set_error(ABACUS_PW_EINTERNAL, "internal error");
    }
}

extern "C" {

int abacus_pw_last_error(char *buf, int size) {
    if (!buf || size <= 0) return (int)t_err.size();
    std::snprintf(buf, (size_t)size, "%s", t_err.c_str());
    return (int)t_err.size();
}

int abacus_pw_fft_supported(int n) { return local_length_supported(n); }

int abacus_pw_plan_reset(void) {
    return guarded([&] { return plan_reset_all(); });
}

int abacus_pw_set_tuning(int band_batch, int splitk_chunk, int yz_bands, int x_bands, int yz_mode, int overlap,
                         int yz_threads) {
    if (band_batch < 0 || splitk_chunk < 0 || yz_bands < 0 || x_bands < 0 || yz_mode < 0 || yz_mode > 2 ||
        overlap < 0 || overlap > 2 || (yz_threads != 0 && yz_threads != 256 && yz_threads != 512 && yz_threads != 1024))
        return set_error(ABACUS_PW_EBAD_SHAPE,
                         "tuning values must be >= 0 (yz_mode and overlap 0, 1 or 2; yz_threads 0, 256, 512 or 1024)");
    g_yz_threads = yz_threads;
    g_yz_mode = yz_mode;
    g_overlap = overlap;
    g_band_batch = band_batch;
    g_splitk_chunk = splitk_chunk;
    g_yz_bands = yz_bands;
    g_x_bands = x_bands;
    return ABACUS_PW_OK;
}

int abacus_pw_profile_enable(int on) {
    g_prof_on = on != 0;
    return ABACUS_PW_OK;
}

int abacus_pw_profile_read(char *buf, int size) {
    return guarded([&]() -> int {
        APW_HIP(hipDeviceSynchronize());
        APW_TRY(prof_collect());
        std::string out;
        int n = 0;
        {
            std::lock_guard<std::mutex> l(g_prof_mu);
            for (auto &kv : g_totals) {
                char line[320];
                std::snprintf(line, sizeof line, "%s\t%ld\t%.6f\t%.6e\n", kv.first.c_str(), kv.second.n,
                              kv.second.ms, kv.second.flops);
                out += line;
                ++n;
            }
            g_totals.clear();
        }
        if (buf && size > 0) std::snprintf(buf, (size_t)size, "%s", out.c_str());
        return n;
    });
}

int abacus_pw_apply_h(const abacus_pw_problem *p, int precision, int nb, const void *psi, void *hpsi, void *stream) {
    return guarded([&]() -> int {
        if (!psi || !hpsi) return set_error(ABACUS_PW_ENULL_ARG, "psi and hpsi are required");
        if (psi == hpsi) return set_error(ABACUS_PW_EBAD_SHAPE, "hpsi must not alias psi");
        if (nb < 1) return set_error(ABACUS_PW_EBAD_SHAPE, "nb must be >= 1");
        if (precision < 0 || precision > 3) return set_error(ABACUS_PW_EBAD_PRECISION, "unknown precision");
        std::shared_ptr<Plan> P;
        APW_TRY(get_plan(p, static_cast<hipStream_t>(stream), P));
        return apply_h_all(*p, *P, precision, nb, psi, hpsi, static_cast<hipStream_t>(stream));
    });
}

int abacus_pw_workspace_size(const abacus_pw_problem *p, int precision, int nb, size_t *bytes, void *stream) {
    return guarded([&]() -> int {
        if (!bytes) return set_error(ABACUS_PW_ENULL_ARG, "bytes is required");
        if (nb < 1) return set_error(ABACUS_PW_EBAD_SHAPE, "nb must be >= 1");
        if (precision < 0 || precision > 3) return set_error(ABACUS_PW_EBAD_PRECISION, "unknown precision");
        std::shared_ptr<Plan> P;
        APW_TRY(get_plan(p, static_cast<hipStream_t>(stream), P));
        return apply_h_workspace(*P, precision, nb, bytes);
    });
}

int abacus_pw_apply_h_ws(const abacus_pw_problem *p, int precision, int nb, const void *psi, void *hpsi,
                         void *workspace, size_t ws_bytes, void *stream) {
    return guarded([&]() -> int {
        if (!psi || !hpsi || !workspace) return set_error(ABACUS_PW_ENULL_ARG, "psi, hpsi and workspace are required");
        if (psi == hpsi) return set_error(ABACUS_PW_EBAD_SHAPE, "hpsi must not alias psi");
        if (nb < 1) return set_error(ABACUS_PW_EBAD_SHAPE, "nb must be >= 1");
        if (precision < 0 || precision > 3) return set_error(ABACUS_PW_EBAD_PRECISION, "unknown precision");
        if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
            return set_error(ABACUS_PW_EBAD_SHAPE, "workspace must be 256-byte aligned");
        std::shared_ptr<Plan> P;
        APW_TRY(get_plan(p, static_cast<hipStream_t>(stream), P));
        return apply_h_all(*p, *P, precision, nb, psi, hpsi, static_cast<hipStream_t>(stream), workspace, ws_bytes);
    });
}

int abacus_pw_apply_h_backward(const abacus_pw_problem *p, int precision, int nb, const void *psi, const void *dY,
                               void *grad_psi, double *grad_vloc, double *grad_dmat, void *stream) {
    return guarded([&]() -> int {
        if (!psi || !dY) return set_error(ABACUS_PW_ENULL_ARG, "psi and dY are required");
        if (nb < 1) return set_error(ABACUS_PW_EBAD_SHAPE, "nb must be >= 1");
        if (precision != ABACUS_PW_FP64 && precision != ABACUS_PW_FP32)
            return set_error(ABACUS_PW_EBAD_PRECISION, "the adjoint runs in FP64 or FP32");
        std::shared_ptr<Plan> P;
        APW_TRY(get_plan(p, static_cast<hipStream_t>(stream), P));
        return apply_h_backward_all(*p, *P, precision, nb, psi, dY, grad_psi, grad_vloc, grad_dmat,
                                    static_cast<hipStream_t>(stream));
    });
}

int abacus_pw_density(const abacus_pw_problem *p, int precision, int nb, const void *psi, const double *occ,
                      double *rho, void *stream) {
    return guarded([&]() -> int {
        if (!psi || !occ || !rho) return set_error(ABACUS_PW_ENULL_ARG, "psi, occ and rho are required");
        if (nb < 1) return set_error(ABACUS_PW_EBAD_SHAPE, "nb must be >= 1");
        if (precision != ABACUS_PW_FP64 && precision != ABACUS_PW_FP32)
            return set_error(ABACUS_PW_EBAD_PRECISION, "the density runs in FP64 or FP32");
        std::shared_ptr<Plan> P;
        APW_TRY(get_plan(p, static_cast<hipStream_t>(stream), P));
        return density_all(*p, *P, precision, nb, psi, occ, rho, static_cast<hipStream_t>(stream));
    });
}

int abacus_pw_force_nl(const abacus_pw_problem *p, int precision, int nb, const void *psi, const double *occ,
                       double *force, void *stream) {
    return guarded([&]() -> int {
        if (!psi || !occ || !force) return set_error(ABACUS_PW_ENULL_ARG, "psi, occ and force are required");
        if (nb < 1) return set_error(ABACUS_PW_EBAD_SHAPE, "nb must be >= 1");
        if (precision != ABACUS_PW_FP64) return set_error(ABACUS_PW_EBAD_PRECISION, "the force runs in FP64");
        std::shared_ptr<Plan> P;
        APW_TRY(get_plan(p, static_cast<hipStream_t>(stream), P));
        return force_nl_all(*p, *P, nb, psi, occ, force, static_cast<hipStream_t>(stream));
    });
}

int abacus_pw_chebyshev(const abacus_pw_problem *p, int precision, int nb, const void *chi, void *out,
                        const double *coef, int order, double emin, double emax, void *stream) {
    return guarded([&]() -> int {
        if (!chi || !out || !coef) return set_error(ABACUS_PW_ENULL_ARG, "chi, out and coef are required");
        if (chi == out) return set_error(ABACUS_PW_EBAD_SHAPE, "out must not alias chi");
        if (nb < 1 || order < 0) return set_error(ABACUS_PW_EBAD_SHAPE, "need nb >= 1 and order >= 0");
        if (!std::isfinite(emin) || !std::isfinite(emax) || !(emax > emin))
            return set_error(ABACUS_PW_EBAD_SHAPE, "need finite emin < emax");
        for (int i = 0; i <= order; ++i)
            if (!std::isfinite(coef[i])) return set_error(ABACUS_PW_ENONFINITE, "coefficient is not finite");
        if (precision < 0 || precision > 3) return set_error(ABACUS_PW_EBAD_PRECISION, "unknown precision");
        std::shared_ptr<Plan> P;
        APW_TRY(get_plan(p, static_cast<hipStream_t>(stream), P));
        return chebyshev_all(*p, *P, precision, nb, chi, out, coef, order, emin, emax,
                             static_cast<hipStream_t>(stream));
    });
}

int abacus_pw_chebyshev_coefficients(int order, double emin, double emax, double mu, double kt, double power,
                                     double *coef) {
    return guarded([&]() -> int {
        if (!coef) return set_error(ABACUS_PW_ENULL_ARG, "coef is required");
        if (order < 0) return set_error(ABACUS_PW_EBAD_SHAPE, "need order >= 0");
        if (!std::isfinite(emin) || !std::isfinite(emax) || !(emax > emin) || !std::isfinite(mu) ||
            !(kt > 0.0) || !std::isfinite(kt) || !(power > 0.0) || !std::isfinite(power))
            return set_error(ABACUS_PW_EBAD_SHAPE, "need finite emin < emax, mu, kt > 0 and power > 0");
        fermi_coefficients(order, emin, emax, mu, kt, power, coef);
        return ABACUS_PW_OK;
    });
}

int abacus_pw_eigh_lowest(int n, void *A, int ld, int nw, double *w, void *vec, int ldv, void *stream) {
    return guarded([&]() -> int {
        if (!A || !w || !vec) return set_error(ABACUS_PW_ENULL_ARG, "A, w and vec are required");
        if (n < 1 || n > kMaxSub || nw < 1 || nw > n || ld < n || ldv < n)
            return set_error(ABACUS_PW_EBAD_SHAPE, "need 1 <= nw <= n <= 4096, ld >= n, ldv >= n");
        void *ws = nullptr;
        int *info = nullptr;
        APW_TRY(dense_workspace(heev_scratch_bytes(n), &ws, &info));
        return heev_lowest(n, static_cast<z64 *>(A), ld, nw, w, static_cast<z64 *>(vec), ldv, ws,
                           static_cast<hipStream_t>(stream));
    });
}

int abacus_pw_cholesky(int n, void *G, int ld, void *Linv, int ldi, void *stream) {
    return guarded([&]() -> int {
        if (!G || !Linv) return set_error(ABACUS_PW_ENULL_ARG, "G and Linv are required");
        if (n < 1 || n > kMaxChol || ld < n || ldi < n)
            return set_error(ABACUS_PW_EBAD_SHAPE, "need 1 <= n <= 1024, ld >= n, ldi >= n");
        void *ws = nullptr;
        int *info = nullptr;
        hipStream_t st = static_cast<hipStream_t>(stream);
        APW_TRY(dense_workspace(potrf_scratch_bytes(n), &ws, &info));
        APW_TRY(potrf_inv(n, static_cast<z64 *>(G), ld, static_cast<z64 *>(Linv), ldi, info, ws, st));
        int h = 0;
        APW_HIP(hipMemcpyAsync(&h, info, sizeof(int), hipMemcpyDeviceToHost, st));
        APW_HIP(hipStreamSynchronize(st));
        if (h != 0)
            return set_error(ABACUS_PW_ECHOLESKY, "matrix is not positive definite (pivot " + std::to_string(h) + ")");
        return ABACUS_PW_OK;
    });
}

int abacus_pw_davidson(const abacus_pw_problem *p, int precision, int nb, void *psi_inout, double *eig, double tol,
                       int max_iter, int ndim, int *iters, double *resid, void *stream) {
    return guarded([&]() -> int {
        if (!psi_inout || !eig) return set_error(ABACUS_PW_ENULL_ARG, "psi_inout and eig are required");
        if (nb < 1 || max_iter < 0 || ndim < 2) return set_error(ABACUS_PW_EBAD_SHAPE, "need nb >= 1, max_iter >= 0, ndim >= 2");
        if (!(tol > 0.0)) return set_error(ABACUS_PW_EBAD_SHAPE, "tol must be > 0");
        if (precision != ABACUS_PW_FP64 && precision != ABACUS_PW_MIXED_FP32 && precision != ABACUS_PW_MIXED_BF16)
            return set_error(ABACUS_PW_EBAD_PRECISION, "Davidson runs in FP64 or a MIXED mode");
        std::shared_ptr<Plan> P;
        APW_TRY(get_plan(p, static_cast<hipStream_t>(stream), P));
        for (int k = 0; k < p->nk; ++k)
            if (p->npw[k] < nb) return set_error(ABACUS_PW_EBAD_SHAPE, "nb exceeds the sphere size");
        return davidson_all(*p, *P, precision, nb, psi_inout, eig, tol, max_iter, ndim, iters, resid,
                            static_cast<hipStream_t>(stream));
    });
}

int abacus_pw_cg(const abacus_pw_problem *p, int nb, void *psi_inout, double *eig, double tol, int max_iter,
                 int *iters, double *resid, void *stream) {
    return guarded([&]() -> int {
        if (!psi_inout || !eig) return set_error(ABACUS_PW_ENULL_ARG, "psi_inout and eig are required");
        if (nb < 1 || max_iter < 0) return set_error(ABACUS_PW_EBAD_SHAPE, "need nb >= 1, max_iter >= 0");
        if (!(tol > 0.0)) return set_error(ABACUS_PW_EBAD_SHAPE, "tol must be > 0");
        std::shared_ptr<Plan> P;
        APW_TRY(get_plan(p, static_cast<hipStream_t>(stream), P));
        for (int k = 0; k < p->nk; ++k)
            if (p->npw[k] < nb) return set_error(ABACUS_PW_EBAD_SHAPE, "nb exceeds the sphere size");
        return cg_all(*p, *P, nb, psi_inout, eig, tol, max_iter, iters, resid, static_cast<hipStream_t>(stream));
    });
}

}  // extern "C"

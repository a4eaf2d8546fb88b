// Chebyshev-filtered application (abacus_pw_chebyshev) and the Fermi-Dirac
// expansion coefficients (abacus_pw_chebyshev_coefficients).
//
// Sec. III.C filters stochastic orbitals by f_H^{1/2}, f_H the Fermi-Dirac
// operator, expanded in Chebyshev polynomials of H mapped onto [-1, 1]. Here
//   out = sum_{n=0}^{M} c_n T_n(Hs) chi,   Hs = (H - c) / h,
//   c = (emax + emin) / 2, h = (emax - emin) / 2,
// by the three-term recurrence T_0 chi = chi, T_1 chi = Hs chi,
// T_{n+1} chi = 2 Hs T_n chi - T_{n-1} chi. Each step is one H psi on all
// bands (the library's apply path) and one fused pass that forms the next
// term from H T_n chi, T_n chi and T_{n-1} chi and adds c_{n+1} times it to out.
#include <cmath>

#include "hamiltonian.hpp"

namespace apw {

namespace {

// next = a hv + b cur (+ g prev); acc += cn next. prev and next may be the same
// array (each element is read before it is written by the same thread).
template <typename T, bool kPrev>
__global__ __launch_bounds__(256) void k_cheb_step(int64_t n, const cx<T> *__restrict__ hv,
                                                   const cx<T> *__restrict__ cur, const cx<T> *prev, cx<T> *next,
                                                   cx<T> *__restrict__ acc, T a, T b, T g, T cn) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const cx<T> h = hv[i], u = cur[i];
        T re = a * h.re + b * u.re, im = a * h.im + b * u.im;
        if (kPrev) {
            const cx<T> w = prev[i];
            re += g * w.re;
            im += g * w.im;
        }
        const cx<T> o = acc[i];
        next[i] = cx<T>{re, im};
        acc[i] = cx<T>{o.re + cn * re, o.im + cn * im};
    }
}

// acc = c0 chi
template <typename T>
__global__ __launch_bounds__(256) void k_cheb_init(int64_t n, const cx<T> *__restrict__ chi, cx<T> *__restrict__ acc,
                                                   T c0) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const cx<T> x = chi[i];
        acc[i] = cx<T>{c0 * x.re, c0 * x.im};
    }
}

unsigned stream_blocks(int64_t n) { return (unsigned)std::min<int64_t>(ceil_div64(n, 256), 8192); }

template <typename T>
int cheb_step(int64_t n, const void *hv, const void *cur, const void *prev, void *next, void *acc, double a, double b,
              double g, double cn, hipStream_t st) {
    KernelTimer kt("cheb_step", st);
    if (prev)
        hipLaunchKernelGGL((k_cheb_step<T, true>), dim3(stream_blocks(n)), dim3(256), 0, st,
                           n, static_cast<const cx<T> *>(hv), static_cast<const cx<T> *>(cur),
                           static_cast<const cx<T> *>(prev), static_cast<cx<T> *>(next), static_cast<cx<T> *>(acc),
                           (T)a, (T)b, (T)g, (T)cn);
    else
        hipLaunchKernelGGL((k_cheb_step<T, false>), dim3(stream_blocks(n)), dim3(256), 0, st,
                           n, static_cast<const cx<T> *>(hv), static_cast<const cx<T> *>(cur),
                           static_cast<const cx<T> *>(cur), static_cast<cx<T> *>(next), static_cast<cx<T> *>(acc),
                           (T)a, (T)b, (T)0, (T)cn);
    return check_launch("cheb_step");
}

template <typename T>
int chebyshev_t(const abacus_pw_problem &p, Plan &P, int prec, int nb, const void *chi, void *out,
                const double *coef, int order, double emin, double emax, hipStream_t st) {
    const int64_t n = (int64_t)nb * P.npw_total;
    const size_t bytes = sizeof(cx<T>) * (size_t)n;
    for (auto &buf : P.cheb) APW_TRY(buf.ensure(bytes));
    const double c = 0.5 * (emax + emin), h = 0.5 * (emax - emin);
    {
        KernelTimer kt("cheb_step", st);
        hipLaunchKernelGGL((k_cheb_init<T>), dim3(stream_blocks(n)), dim3(256), 0, st, n,
                           static_cast<const cx<T> *>(chi), static_cast<cx<T> *>(out), (T)coef[0]);
        APW_TRY(check_launch("cheb_init"));
    }
    if (order == 0) return ABACUS_PW_OK;
    void *hv = P.cheb[2].ptr;
    // T_1 chi = (H chi - c chi) / h
    APW_TRY(apply_h_all(p, P, prec, nb, chi, hv, st));
    APW_TRY(cheb_step<T>(n, hv, chi, nullptr, P.cheb[0].ptr, out, 1.0 / h, -c / h, 0.0, coef[1], st));
    const void *prev = chi;
    void *cur = P.cheb[0].ptr;
    for (int m = 2; m <= order; ++m) {
        APW_TRY(apply_h_all(p, P, prec, nb, cur, hv, st));
        // the term two back is overwritten in place, except the caller's chi
        void *next = prev == chi ? P.cheb[1].ptr : const_cast<void *>(prev);
        APW_TRY(cheb_step<T>(n, hv, cur, prev, next, out, 2.0 / h, -2.0 * c / h, -1.0, coef[m], st));
        prev = cur;
        cur = next;
    }
    return ABACUS_PW_OK;
}

}  // namespace

int chebyshev_all(const abacus_pw_problem &p, Plan &P, int prec, int nb, const void *chi, void *out,
                  const double *coef, int order, double emin, double emax, hipStream_t st) {
    return prec == ABACUS_PW_FP32 ? chebyshev_t<float>(p, P, prec, nb, chi, out, coef, order, emin, emax, st)
                                  : chebyshev_t<double>(p, P, prec, nb, chi, out, coef, order, emin, emax, st);
}

// Chebyshev interpolation of g(E) = f(E)^power on [emin, emax] at the M + 1
// Chebyshev points of the first kind x_j = cos(pi (j + 1/2) / (M + 1)):
//   c_n = (2 - [n == 0]) / (M + 1) sum_j g(c + h x_j) cos(n pi (j + 1/2) / (M + 1)),
// the discrete orthogonality of T_n on those points; f = 1 / (1 + exp(z)),
// z = (E - mu) / kt, evaluated as exp(-z) / (1 + exp(-z)) for z > 0 so that its
// tail keeps full relative precision.
void fermi_coefficients(int order, double emin, double emax, double mu, double kt, double power, double *coef) {
    const int M1 = order + 1;
    const double c = 0.5 * (emax + emin), h = 0.5 * (emax - emin);
    std::vector<double> g(M1);
    for (int j = 0; j < M1; ++j) {
        const double x = std::cos(M_PI * (j + 0.5) / M1);
        const double z = (c + h * x - mu) / kt;
        const double f = z > 0.0 ? std::exp(-z) / (1.0 + std::exp(-z)) : 1.0 / (1.0 + std::exp(z));
        g[j] = std::pow(f, power);
    }
    // the angle pi n (2j + 1) / (2 (M + 1)) is reduced modulo 2 pi in integers first
    const int64_t period = 4 * (int64_t)M1;
    for (int n = 0; n < M1; ++n) {
        double s = 0.0;
        for (int j = 0; j < M1; ++j) {
            const int64_t t = ((int64_t)n * (2 * j + 1)) % period;
            s += g[j] * std::cos(M_PI * (double)t / (2.0 * M1));
        }
        coef[n] = (n == 0 ? 1.0 : 2.0) * s / M1;
    }
}

}  // namespace apw

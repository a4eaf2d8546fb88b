// Drivers behind the C entry points.
#pragma once

#include "plan.hpp"

namespace apw {

int default_band_batch(const Plan &P, int nb);
int operator_copies(const abacus_pw_problem &p, Plan &P, bool need_v32, bool need_b32, hipStream_t st,
                    bool need_bf = false);

// hpsi = H psi for nb bands of k-point k ([nb][npw_k] blocks). refresh_copies re-derives the
// reduced-precision copies of V and beta (unless the problem is flagged static).
int apply_h_k(const abacus_pw_problem &p, Plan &P, int k, int prec, int nb, const void *psi, void *hpsi,
              hipStream_t st, bool refresh_copies = true);

// Per-call work buffers of H psi: slab, Q, split-K partials, bf16 psi, bf16 Q, FP32 psi.
constexpr int kHWorkParts = 6;

// hpsi = H psi for nb bands at the k-points [k0, k1) (psi starts at k0's block). The work
// buffers come from the plan (grown as needed) unless ws (ws_bytes) is given, in which case
// they are carved from it and nothing is allocated.
int apply_h_range(const abacus_pw_problem &p, Plan &P, int k0, int k1, int prec, int nb, const void *psi, void *hpsi,
                  hipStream_t st, bool refresh_copies, void *ws = nullptr, size_t ws_bytes = 0);

// hpsi = H psi for nb bands at every k-point (packed [k][nb][npw_k]).
int apply_h_all(const abacus_pw_problem &p, Plan &P, int prec, int nb, const void *psi, void *hpsi, hipStream_t st,
                void *ws = nullptr, size_t ws_bytes = 0);

// Bytes of caller work space apply_h_all needs for (prec, nb) with the current knobs; allocates
// the plan's operator copies for prec (and the side stream when the overlap knob is on) so a
// later call with that work space allocates nothing.
int apply_h_workspace(Plan &P, int prec, int nb, size_t *bytes);

// Adjoint of apply_h_all (abacus_pw_apply_h_backward).
int apply_h_backward_all(const abacus_pw_problem &p, Plan &P, int prec, int nb, const void *psi, const void *dy,
                         void *grad_psi, double *grad_v, double *grad_d, hipStream_t st);
// Band density rho(r_j) = sum_{k,n} occ[k][n] |psi_nk(r_j)|^2 (occ device [nk][nb]); rho overwritten.
int density_all(const abacus_pw_problem &p, Plan &P, int prec, int nb, const void *psi, const double *occ,
                double *rho, hipStream_t st);

// out = sum_{n<=order} coef[n] T_n((H - c)/h) chi, c and h the centre and half width of
// [emin, emax]; coef is host memory, read during the call.
// Nonlocal force F[natom][3] (Ry/bohr) = -dE_NL/dtau with E_NL = sum_{k,n} occ[k][n] <psi|V_NL|psi>;
// occ device [nk][nb]; force device, overwritten. FP64.
int force_nl_all(const abacus_pw_problem &p, Plan &P, int nb, const void *psi, const double *occ, double *force,
                 hipStream_t st);
int chebyshev_all(const abacus_pw_problem &p, Plan &P, int prec, int nb, const void *chi, void *out,
                  const double *coef, int order, double emin, double emax, hipStream_t st);
// Chebyshev interpolation coefficients [order + 1] of the Fermi-Dirac function to a power.
void fermi_coefficients(int order, double emin, double emax, double mu, double kt, double power, double *coef);

// Band-by-band preconditioned CG (abacus_pw_cg).
int cg_all(const abacus_pw_problem &p, Plan &P, int nb, void *psi, double *eig, double tol, int max_iter, int *iters,
           double *resid, hipStream_t st);

// Block Davidson (abacus_pw_davidson).
int davidson_all(const abacus_pw_problem &p, Plan &P, int prec, int nb, void *psi, double *eig, double tol,
                 int max_iter, int ndim, int *iters, double *resid, hipStream_t st);

}  // namespace apw

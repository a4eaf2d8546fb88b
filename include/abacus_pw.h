/*
 * abacus_pw.h -- C ABI of the MI355X (gfx950) plane-wave Hamiltonian library.
 *
 * The library applies the Kohn-Sham Hamiltonian of the plane-wave method
 * (Sec. III.A, the KS equation written in the plane-wave basis) to blocks of
 * bands, and solves for its lowest eigenpairs with a block Davidson method
 * (Sec. III.B names Davidson as the iterative eigensolver) or band-by-band CG
 * (the CG figure of Sec. III.B). Around that it provides the adjoint of H psi,
 * the band density, the Chebyshev-filtered application of Sec. III.C and the
 * nonlocal force of Sec. III.A. The potential is
 * the norm-conserving split of Sec. II.A ("Pseudopotentials"): a local part
 * sampled on the real-space FFT grid plus the Kleinman-Bylander separable
 * nonlocal part sum_ij |beta_i> D_ij <beta_j|.
 *
 * Units: Rydberg atomic units. Energies in Ry, lengths in bohr; the kinetic
 * operator is |k+G|^2 (the paper's Hartree form is (1/2)|k+G|^2).
 *
 * Conventions used by every entry point:
 *   - A k-point's basis is its G-sphere S_k = {G = sum_i m_i b_i : |k+G|^2 < ecutwfc},
 *     given by the caller as Miller triples (m1, m2, m3) in any order; that
 *     order is the order of every coefficient array.
 *   - Real-space grid r_j = sum_i (j_i / N_i) a_i, stored C-ordered [N1][N2][N3]
 *     (j3 fastest). A Miller index m maps to grid index m mod N_i.
 *   - psi(r_j) = sum_G psi(G) e^{+iG.r_j} (unnormalised) and
 *     (V psi)(G) = (1/N) sum_j e^{-iG.r_j} V(r_j) psi(r_j), N = N1 N2 N3; the
 *     1/N is the grid form of the density transform rho(G) = (1/Omega) int
 *     rho(r) e^{-iG.r} dr of Sec. III.A.
 *   - So (H psi)(G) = |k+G|^2 psi(G) + sum_{G'} Vt((m-m') mod N) psi(G')
 *                     + sum_ij beta_i(G) D_ij <beta_j|psi>,
 *     with Vt(q) = (1/N) sum_j V(r_j) e^{-2 pi i q.j/N}. Differences G-G'
 *     wrap modulo the grid, as on any finite FFT grid.
 *   - Inner products are coefficient sums <x|y> = sum_G conj(x(G)) y(G);
 *     "orthonormal" means Psi^H Psi = I in that product.
 *   - Complex arrays are interleaved (re, im): complex128 = two doubles,
 *     complex64 = two floats, the layout of torch.complex128 / complex64.
 *   - Band arrays (psi, H psi, gradients) are packed k-major: for each k a
 *     [nb][npw_k] block, blocks back to back.
 *
 * Memory and streams: the caller owns every buffer it passes and the library
 * never frees caller memory. Device pointers must be device memory of the
 * current HIP device. `stream` is a hipStream_t (NULL = the null stream); all
 * device work is enqueued on it. The library keeps a per-process plan cache
 * (geometry tables, work space) keyed by the problem's geometry; the first call
 * for a geometry builds the plan (it allocates and synchronises), later calls
 * only enqueue kernels.
 *
 * Threads: the plan cache is shared and locked; a plan evicted by one thread
 * stays alive until every call that holds it has returned, and its device
 * buffers are freed only after the device is idle. Calls that share a plan
 * (same geometry) share its work space: they must be issued on one stream, or
 * the caller must order them (events, synchronisation). Calls on different
 * plans are independent. The tuning knobs (abacus_pw_set_tuning) are
 * process-wide.
 *
 * Errors: every entry point returns 0 on success and a negative ABACUS_PW_E*
 * code on failure (nothing has been enqueued when a validation error is
 * returned); abacus_pw_last_error() gives a message for the calling thread.
 * No C++ exception crosses this interface.
 */
#ifndef ABACUS_PW_H
#define ABACUS_PW_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define ABACUS_PW_OK                    0
#define ABACUS_PW_NOT_CONVERGED         1   /* Davidson hit max_iter; outputs are valid */
#define ABACUS_PW_ENULL_ARG            -1   /* a required pointer is NULL */
#define ABACUS_PW_EBAD_SHAPE           -2   /* nk, npw, nb, nproj, natom or offsets inconsistent */
#define ABACUS_PW_EBAD_FFT_SIZE        -3   /* a grid length is unsupported, or 2 max|m_i| + 1 > N_i */
#define ABACUS_PW_EBAD_SPHERE          -4   /* duplicate Miller triple, or |k+G|^2 >= ecutwfc */
#define ABACUS_PW_EBAD_D               -5   /* a D block is not symmetric (1e-14 relative) */
#define ABACUS_PW_ENONFINITE           -6   /* NaN/Inf in V_loc or D */
#define ABACUS_PW_EBAD_PRECISION       -7   /* unknown precision value, or mode not offered by this entry point */
#define ABACUS_PW_EHIP                 -8   /* a HIP runtime call failed */
#define ABACUS_PW_ECHOLESKY            -9   /* Davidson: Gram matrix not positive definite even after a shift */
#define ABACUS_PW_EINTERNAL           -10

/* Arithmetic modes (the `precision` argument). */
#define ABACUS_PW_FP64        0  /* complex128 psi; FP64 FFTs and GEMMs */
#define ABACUS_PW_FP32        1  /* complex64 psi; FP32 FFTs and FP32-MFMA GEMMs with FP32 accumulation */
#define ABACUS_PW_MIXED_BF16  2  /* complex128 psi in and out; FP32 FFTs; BF16 projector GEMM operands, FP32 accumulation */
#define ABACUS_PW_MIXED_FP32  3  /* complex128 psi in and out; FP32 FFTs; FP32 GEMM operands, FP32 accumulation */

/* problem.flags */
#define ABACUS_PW_STATIC_OPERATOR 1u  /* V_loc, beta and D contents are unchanged since the last call
                                         with the same pointers: reduced-precision copies may be reused */

/*
 * The problem statement (the plane-wave KS problem of Sec. III.A with the
 * pseudopotential split of Sec. II.A).
 *
 * lattice          host, rows a1, a2, a3 (bohr).
 * fft              N1, N2, N3: grid lengths; each must be a product of 2, 3 and 5
 *                  that the library has a transform for (see abacus_pw_fft_supported).
 * ecutwfc          kinetic cutoff (Ry); every sphere point must satisfy |k+G|^2 < ecutwfc.
 * nk, kpts         host [nk][3] cartesian k-points (bohr^-1).
 * npw              host [nk] sphere sizes.
 * miller           host [sum npw][3] int32 Miller triples, k-major (the G-sphere index map).
 *                  The plan cache keys on the pointer and a hash of every triple, so a map
 *                  edited in place gets a new plan.
 * vloc             device [N1][N2][N3] float64 local potential V_loc(r_j) (Ry).
 * nproj            projectors per k-point (same count and order at every k).
 * natom            number of atom blocks.
 * proj_atom_offset host [natom+1]: projectors of atom a are [off[a], off[a+1]).
 * beta             device complex128, per k a [nproj][npw_k] block of beta_i(k+G).
 * dmat             device float64, per atom a row-major [np_a][np_a] symmetric block of D (Ry),
 *                  blocks back to back.
 * flags            ABACUS_PW_STATIC_OPERATOR or 0.
 *
 * V_loc and D are checked (finite; D symmetric) once per plan, when the plan is
 * first built, by copies enqueued on the caller's stream (so they see the
 * caller's earlier writes). Later calls with the same geometry reuse the plan
 * and do not re-check: a caller that changes V or D between calls (an SCF
 * update, a finite-difference step) is responsible for their finiteness and
 * for the symmetry of D.
 */
typedef struct abacus_pw_problem {
    double lattice[9];
    int fft[3];
    double ecutwfc;
    int nk;
    const double *kpts;
    const int *npw;
    const int *miller;
    const double *vloc;
    int nproj;
    int natom;
    const int *proj_atom_offset;
    const void *beta;
    const double *dmat;
    unsigned flags;
} abacus_pw_problem;

/*
 * hpsi = H psi for nb bands at every k-point (KS equation in the plane-wave
 * basis, Sec. III.A; local + Kleinman-Bylander terms, Sec. II.A).
 *
 * psi   device, packed [k][nb][npw_k]: complex128 for FP64 and MIXED_*, complex64 for FP32.
 * hpsi  device, same layout and type as psi; overwritten. Must not alias psi.
 * Asynchronous: returns after enqueueing on `stream` (after the plan exists).
 * Errors: ENULL_ARG, EBAD_SHAPE, EBAD_FFT_SIZE, EBAD_SPHERE, EBAD_D, ENONFINITE,
 * EBAD_PRECISION, EHIP.
 */
int abacus_pw_apply_h(const abacus_pw_problem *p, int precision, int nb, const void *psi, void *hpsi,
                      void *stream);

/*
 * H psi with a work space supplied by the caller (the hpsi = H psi of
 * abacus_pw_apply_h, Sec. III.A / II.A, same results bit for bit).
 *
 * abacus_pw_workspace_size builds the problem's plan if it does not exist (it
 * allocates the plan's tables and its reduced-precision operator copies for
 * `precision`, and synchronises) and writes to *bytes the work-space size
 * abacus_pw_apply_h_ws needs for nb bands at that precision: the slab of
 * grid planes of one band batch at every k-point, the projections and their
 * split-K partial sums (and the bf16 / FP32 staging of the mixed modes). The
 * size depends on the tuning knobs (band batch, split-K chunk): query it again
 * after abacus_pw_set_tuning.
 *
 * abacus_pw_apply_h_ws then applies H using `workspace` (device memory of at
 * least that many bytes, 256-byte aligned, owned by the caller; its contents are
 * scratch). Once the plan exists, the call allocates nothing, synchronises
 * nothing and records no memset, so even its first call can be captured in a
 * HIP graph. Calls sharing one work space must be ordered by the caller.
 * Errors: those of abacus_pw_apply_h, ENULL_ARG (workspace), EBAD_SHAPE (work space too
 * small for the current knobs, or misaligned).
 */
int abacus_pw_workspace_size(const abacus_pw_problem *p, int precision, int nb, size_t *bytes, void *stream);
int abacus_pw_apply_h_ws(const abacus_pw_problem *p, int precision, int nb, const void *psi, void *hpsi,
                         void *workspace, size_t ws_bytes, void *stream);

/*
 * Lowest nb eigenpairs of H at every k-point by band-by-band preconditioned
 * conjugate gradients (the CG figure of Sec. III.B): band i is projected
 * against bands 0..i-1 and normalised, then repeatedly moved along a
 * Polak-Ribiere direction built from the Teter-Payne-Allan preconditioned
 * residual (projected against bands 0..i), by the rotation that minimises its
 * Rayleigh quotient, until ||H psi_i - eps_i psi_i|| < tol or max_iter steps.
 * H is applied to one band at a time, in FP64.
 *
 * psi_inout device complex128 packed [k][nb][npw_k]: initial guess in, eigenvectors out
 *           (orthonormal).
 * eig       host float64 [nk][nb]: eigenvalues in band order (Ry).
 * tol       residual tolerance per band.
 * max_iter  maximum number of CG steps per band.
 * iters     host int [nk][nb] (may be NULL): CG steps taken by each band.
 * resid     host float64 [nk][nb] (may be NULL): final residual norms.
 * Returns 0 when every band converged, ABACUS_PW_NOT_CONVERGED (+1) otherwise
 * (outputs valid), or a negative code (ENULL_ARG, EBAD_SHAPE, EBAD_FFT_SIZE,
 * EBAD_SPHERE, EBAD_D, ENONFINITE, EHIP). Synchronises `stream` before returning.
 */
int abacus_pw_cg(const abacus_pw_problem *p, int nb, void *psi_inout, double *eig, double tol, int max_iter,
                 int *iters, double *resid, void *stream);

/*
 * Lowest nb eigenpairs of H at every k-point by block Davidson (Sec. III.B
 * names Davidson as the eigensolver of the plane-wave code without its steps;
 * the steps below are the library's): residuals R = H Psi - Psi Lambda,
 * Teter-Payne-Allan preconditioned corrections for unconverged bands, two
 * classical Gram-Schmidt passes against the locked vectors and the basis,
 * Cholesky-QR, Rayleigh-Ritz on the basis [Psi, T]. When the basis would exceed
 * ndim*nb columns it restarts from the Ritz vectors, and the bands already
 * below tol are locked: their pairs are frozen and leave the Rayleigh-Ritz
 * problem, which then keeps the lowest nb - (locked) pairs.
 *
 * psi_inout device complex128 packed [k][nb][npw_k]: initial guess in, Ritz vectors out
 *           (orthonormal).
 * eig       host float64 [nk][nb]: Ritz values, ascending (Ry).
 * tol       residual tolerance: stop when every ||H psi_n - eps_n psi_n||_2 < tol.
 * max_iter  maximum number of correction steps per k-point.
 * ndim      basis size factor (>= 2).
 * iters     host int [nk] (may be NULL): correction steps taken.
 * resid     host float64 [nk][nb] (may be NULL): final residual norms, computed in FP64.
 * precision ABACUS_PW_FP64, or ABACUS_PW_MIXED_FP32 / ABACUS_PW_MIXED_BF16: reduced-precision
 *           Davidson steps followed by FP64 refinement steps to the same tol.
 * Returns 0 when every k converged, ABACUS_PW_NOT_CONVERGED (+1) when max_iter was
 * reached (outputs valid), or a negative code. Synchronises `stream` before returning.
 */
int abacus_pw_davidson(const abacus_pw_problem *p, int precision, int nb, void *psi_inout, double *eig,
                       double tol, int max_iter, int ndim, int *iters, double *resid, void *stream);

/*
 * The dense FP64 steps of the Davidson iteration (Sec. III.B), callable on
 * their own. Matrices are device complex128, row-major with a leading
 * dimension; all work is enqueued on `stream`.
 *
 * abacus_pw_eigh_lowest: the lowest nw eigenpairs of the Hermitian n x n matrix
 * A (both triangles stored; destroyed): Householder reduction to a real
 * tridiagonal matrix, bisection on Sturm counts, inverse iteration, and the
 * back-transformation. n <= 256 runs on one compute unit; larger orders reduce
 * one column at a time with the matrix-vector product spread over the GPU and
 * the rank-2k updates and the back-transformation on the matrix cores.
 *   w     device float64 [nw], ascending.
 *   vec   device complex128 [nw][ldv]: row j is the eigenvector of w[j] (unit norm; vectors of
 *         eigenvalues closer than 1e-7 ||A|| are orthogonalised together, others are
 *         orthogonal to about 1e-16 ||A|| / gap).
 *   Limits 1 <= nw <= n <= 4096, ld >= n, ldv >= n. Asynchronous. Errors: ENULL_ARG, EBAD_SHAPE, EHIP.
 *
 * abacus_pw_cholesky: G = L L^H for a Hermitian positive definite n x n G; the lower triangle
 * of G (diagonal included) is replaced by L, Linv (device [n][ldi]) receives L^{-1} (zero
 * above the diagonal). n <= 136 factors in one work-group's LDS; larger orders in blocks of
 * 64 columns (diagonal block in LDS, panel and trailing update on the matrix cores).
 *   Limits 1 <= n <= 1024. Synchronises `stream`; returns ECHOLESKY when a pivot is not positive.
 *
 * Both hold a work space per device that the library allocates on first use and grows as
 * needed (a call that grows it synchronises the device); calls that overlap on one device
 * share it and must be ordered by the caller (one stream).
 */
int abacus_pw_eigh_lowest(int n, void *A, int ld, int nw, double *w, void *vec, int ldv, void *stream);
int abacus_pw_cholesky(int n, void *G, int ld, void *Linv, int ldi, void *stream);

/*
 * Adjoint of hpsi = H psi for a real loss L with upstream gradient
 * dY = dL/dRe(hpsi) + i dL/dIm(hpsi) (PyTorch's convention for complex tensors):
 *   grad_psi    = H dY                                   (H is Hermitian)
 *   grad_vloc(r_j) = (1/N) sum_{k,n} Re( conj(gamma_n(r_j)) psi_n(r_j) ),
 *                 gamma_n, psi_n the unnormalised inverse transforms of dY_n, psi_n
 *   grad_dmat[a](i,j) = Re sum_{k,n} Q_in conj(P_jn),  P = B^H psi, Q = B^H dY
 * psi, dY   device, layout and type as in abacus_pw_apply_h (FP64 or FP32 precision).
 * grad_psi  device, like psi, overwritten (NULL: skipped).
 * grad_vloc device float64 [N1][N2][N3], overwritten (NULL: skipped).
 * grad_dmat device float64, layout of dmat, overwritten, not symmetrised (NULL: skipped).
 * Reductions over bands and k run in a fixed order (repeatable bit for bit).
 * Asynchronous. Errors as for abacus_pw_apply_h.
 */
int abacus_pw_apply_h_backward(const abacus_pw_problem *p, int precision, int nb, const void *psi,
                               const void *dY, void *grad_psi, double *grad_vloc, double *grad_dmat,
                               void *stream);

/*
 * Band density on the FFT grid. Sec. III.C forms the plane-wave density as a
 * k-weighted sum, over orbitals, of the squared modulus of each orbital's
 * real-space values (the e^{ik.r} factor has modulus one):
 *   rho(r_j) = sum_{k,n} occ[k][n] |psi_nk(r_j)|^2,
 *   psi_nk(r_j) = sum_{G in S_k} c_nk(G) exp(+i G.r_j)   (unnormalised inverse transform,
 *                 Miller index m -> m mod N, no 1/Omega).
 * psi       device, layout and type as in abacus_pw_apply_h (FP64: complex128; FP32: complex64,
 *           with FP32 transforms and FP64 accumulation of the squared moduli).
 * occ       device float64 [nk][nb]: weight of each band (k-point weight times occupation,
 *           spin factor included); any real values.
 * rho       device float64 [N1][N2][N3], overwritten.
 * The sum over bands and k runs in a fixed order (repeatable bit for bit).
 * Asynchronous. Errors: ENULL_ARG, EBAD_SHAPE, EBAD_PRECISION (MIXED modes), and those of
 * abacus_pw_apply_h.
 */
int abacus_pw_density(const abacus_pw_problem *p, int precision, int nb, const void *psi, const double *occ,
                      double *rho, void *stream);

/*
 * Density transform of Sec. III.A on the grid: the reciprocal-space density
 *   rho(G) = (1/N) sum_j rho(r_j) exp(-i G.r_j),   N = N1 N2 N3,
 * the grid form of rho(G) = (1/Omega) int rho(r) e^{-iG.r} dr, for a real density
 * on the grid (for example the output of abacus_pw_density). No plan is needed.
 * fft       host int[3]: N1, N2, N3, each a length with a transform (abacus_pw_fft_supported).
 * rho       device float64 [N1][N2][N3].
 * ng        number of G vectors wanted.
 * miller_g  device int32 [ng][3] Miller triples of the wanted G (for example the density sphere
 *           |G|^2 < 4 ecutwfc). Any integers: a triple is read modulo the grid, so a G outside
 *           the alias-free range 2|m_i| < N_i gets the value of its grid image. NULL: the whole
 *           grid; then ng must equal N and rhog[(i1 N2 + i2) N3 + i3] holds the G with m = i mod N.
 * rhog      device complex128 [ng], overwritten.
 * Work space: with a G list, one complex128 grid (16 N bytes) per device, allocated by the
 * library on first use and grown as needed (a call that grows it synchronises the device);
 * calls with a G list that overlap on one device share it and must be ordered by the caller
 * (one stream). Without a G list the transform runs in rhog itself.
 * Asynchronous. Errors: ENULL_ARG, EBAD_SHAPE (ng < 0; ng != N without a list), EBAD_FFT_SIZE, EHIP.
 */
int abacus_pw_density_g(const int *fft, const double *rho, int ng, const int *miller_g, void *rhog, void *stream);

/*
 * abacus_pw_density_g for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc. Same arguments, kernels and results as abacus_pw_density_g; with a
 * G list the work grid is a fixed device array of the library (2,097,152
 * complex128 points = 32 MiB, the 128^3 grid, one copy per device, held until
 * the process ends) instead of an allocated one. This entry point calls no
 * hipMalloc or hipFree. Every call on a device shares that device's array and
 * leaves its contents behind: calls that overlap on one device (different
 * streams or threads) race and must be ordered by the caller.
 * Errors: as abacus_pw_density_g, plus EBAD_SHAPE for a G list on a grid of more
 * than 2,097,152 points.
 */
int abacus_pw_density_g_noalloc(const int *fft, const double *rho, int ng, const int *miller_g, void *rhog,
                                void *stream);

/*
 * Nonlocal (Kleinman-Bylander) force on every atom, the derivative of the
 * projector energy with respect to the atomic positions (Sec. III.A). With the
 * projectors carrying the structure factor exp(-i (k+G).tau_a):
 *   E_NL = sum_k sum_n occ[k][n] sum_a P_a^H D_a P_a,  P = B^H psi,
 *   F[a][alpha] = -dE_NL/dtau_{a,alpha}
 *               = -2 sum_k sum_n occ[k][n] sum_{i,j in a} D_ij Im(conj(P^alpha_in) P_jn),
 *   P^alpha = B^H ((k+G)_alpha psi),  (k+G) Cartesian in bohr^-1.
 * psi       device complex128 packed [k][nb][npw_k] (FP64 only).
 * occ       device float64 [nk][nb]: weight of each band (k weight x occupation x spin).
 * force     device float64 [natom][3], Ry / bohr, overwritten.
 * At most 16 projectors per atom. Sums over bands and k run in a fixed order.
 * Asynchronous. Errors: ENULL_ARG, EBAD_SHAPE, EBAD_PRECISION (not FP64), and those
 * of abacus_pw_apply_h.
 */
int abacus_pw_force_nl(const abacus_pw_problem *p, int precision, int nb, const void *psi, const double *occ,
                       double *force, void *stream);

/*
 * Chebyshev-filtered application. Sec. III.C applies f_H^{1/2} (f_H the
 * Fermi-Dirac operator) to stochastic orbitals through a Chebyshev expansion
 * in H mapped onto [-1, 1]. This computes, for any coefficients,
 *   out = sum_{n=0}^{order} coef[n] T_n(Hs) chi,  Hs = (H - c) / h,
 *   c = (emax + emin) / 2, h = (emax - emin) / 2,
 * with the three-term recurrence T_{n+1} = 2 Hs T_n - T_{n-1}: `order` applications
 * of H to all nb bands. The expansion converges only when the spectrum of H lies
 * in [emin, emax]; the library does not check this.
 * chi, out  device, layout and type as in abacus_pw_apply_h (out must not alias chi);
 *           out is overwritten.
 * coef      host float64 [order + 1], read before the call returns.
 * precision as in abacus_pw_apply_h; FP32 runs the recurrence in complex64, the other
 *           modes in complex128 with H in that mode's precision.
 * The library holds three work vectors of nb * sum(npw) complex values per plan.
 * Asynchronous. Errors: ENULL_ARG, EBAD_SHAPE (order < 0, emax <= emin, aliasing),
 * ENONFINITE (coefficients), and those of abacus_pw_apply_h.
 */
int abacus_pw_chebyshev(const abacus_pw_problem *p, int precision, int nb, const void *chi, void *out,
                        const double *coef, int order, double emin, double emax, void *stream);

/*
 * Host routine: coefficients coef[0..order] of the degree-`order` Chebyshev
 * interpolant on [emin, emax] of g(E) = f(E)^power, f(E) = 1 / (1 + exp((E - mu) / kt))
 * the Fermi-Dirac function of Sec. III.C (power 1/2 gives the filter f_H^{1/2}),
 * interpolated at the order + 1 Chebyshev points of the first kind. For use with
 * abacus_pw_chebyshev and the same emin, emax. No device access.
 * Errors: ENULL_ARG, EBAD_SHAPE (order < 0, emax <= emin, kt <= 0, power <= 0, non-finite).
 */
int abacus_pw_chebyshev_coefficients(int order, double emin, double emax, double mu, double kt, double power,
                                     double *coef);

/* Message for the last error on the calling thread (truncated to size). Returns len. */
int abacus_pw_last_error(char *buf, int size);

/* 1 when the library has a transform of length n (a product of 2, 3, 5), else 0. */
int abacus_pw_fft_supported(int n);

/* Drops every cached plan (frees their device work space). Synchronises the device. */
int abacus_pw_plan_reset(void);

/*
 * Optional per-kernel timing. When enabled, the library records a pair of HIP
 * events around every kernel it enqueues, on the stream it enqueues it on, and
 * accumulates elapsed time per kernel name at the next abacus_pw_profile_read.
 * abacus_pw_profile_read synchronises, then writes the records
 * "name\tlaunches\ttotal_ms\tflops\n" into buf (NUL-terminated, truncated to size);
 * returns the number of records, or a negative code. Kernels enqueued by the Davidson
 * solver for its subspace (projections, orthogonalisation, Ritz updates, Cholesky-QR and
 * Rayleigh-Ritz products) are named "subspace:<kernel>" and carry their flop count
 * (complex products as 8 M N K); other records carry 0 flops.
 */
int abacus_pw_profile_enable(int on);
int abacus_pw_profile_read(char *buf, int size);

/*
 * Tuning knobs, process-wide (the autotuner sets these; 0 = library default).
 * band_batch   bands per local-term batch (slab work space = band_batch planes sets)
 * splitk_chunk K chunk of the split-K projection GEMM (multiple of 16)
 * yz_bands     bands handled by one y-z plane work-group
 * x_bands      bands handled by one x-pass work-group
 * yz_mode      y-z plane kernels: 0 automatic (whole plane in LDS when it fits), 1 whole
 *              plane, 2 compact (only the plane's z-column rows in LDS, y transforms in
 *              j3 chunks); planes that do not fit whole always use the compact form
 * overlap      0 default (2), 1 the projector GEMMs run on a second stream of the library
 *              (default priority) beside the local term: the projections from the start,
 *              each band batch's B Q as soon as its local term is done; events order the
 *              two streams and join the second back into the caller's stream before the
 *              call returns, so stream semantics and graph capture are unchanged; 2 one stream
 * yz_threads   threads per work-group of the compact-row plane kernels (planes too large
 *              for LDS, one or two work-groups per CU): 256, 512 or 1024 for both passes; 0 =
 *              library default: 512 for the inverse pass, and for the forward pass a form whose
 *              first transform phase loads the slab itself (512 threads) where that phase has
 *              128 to 512 tasks, else 1024
 * Results do not depend on the knobs beyond rounding (the split-K chunk changes the
 * summation grouping of the projections). Returns EBAD_SHAPE for invalid values.
 */
int abacus_pw_set_tuning(int band_batch, int splitk_chunk, int yz_bands, int x_bands, int yz_mode, int overlap,
                         int yz_threads);

#ifdef __cplusplus
}
#endif

#endif /* ABACUS_PW_H */

/*
 * FP64 CPU oracle for the plane-wave Hamiltonian application H psi and its
 * adjoint.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library. The GPU library shares no
 * code, header, table or helper with it.
 *
 * What is computed (Rydberg units, kinetic = |k+G|^2):
 *   Sec. III.A, KS equation in the plane-wave basis:
 *     (H psi)(G) = |k+G|^2 psi(G) + sum_{G'} V(G-G') psi(G') + V_KB psi
 *   Sec. II.A, Kleinman-Bylander separable form:
 *     V_KB = sum_{ij} |beta_i> D_ij <beta_j|, D block-diagonal per atom.
 *   The local term is evaluated on the real-space grid r_j = sum_i (j_i/N_i) a_i:
 *     psi(r_j) = sum_G psi(G) e^{+iG.r_j}          (inverse transform, unnormalised)
 *     (V psi)(G) = (1/N) sum_j e^{-iG.r_j} V(r_j) psi(r_j)
 *   The 1/N forward normalisation is the grid version of the density
 *   transform rho(G) = (1/Omega) int rho(r) e^{-iG.r} dr of Sec. III.A.
 *
 * Everything is plain loops in double / double complex; no blocking, fusion
 * or reordering beyond the definitions above. OpenMP only splits independent
 * bands over threads.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef double complex cplx;

static const double TWO_PI = 6.283185307179586476925286766559;

/* ---------------------------------------------------------------------- */
/* One-dimensional DFT, own implementation.                                */
/* ---------------------------------------------------------------------- */

/* exp(sign * 2 pi i e / n), with the exponent reduced modulo n first. */
static cplx root_of_unity(long e, long n, int sign)
{
    e %= n;
    if (e < 0) e += n;
    double ang = TWO_PI * (double)e / (double)n;
    return cos(ang) + (double)sign * I * sin(ang);
}

static int smallest_factor(int n)
{
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* Direct O(n^2) DFT: y[k] = sum_j x[j*s] exp(sign 2 pi i jk/n). */
void oracle_dft1d(int n, int sign, const cplx *x, long s, cplx *y)
{
    for (int k = 0; k < n; ++k) {
        cplx acc = 0.0;
        for (int j = 0; j < n; ++j)
            acc += x[(long)j * s] * root_of_unity((long)j * k, n, sign);
        y[k] = acc;
    }
}

/*
 * Mixed-radix decimation in time. With n = p*m (p the smallest prime factor)
 * and j = p*t + r:
 *   y[q + m*u] = sum_{r<p} w_n^{r (q + m u)} Y_r[q],
 *   Y_r[q]     = sum_{t<m} x[(p t + r) s] w_m^{t q},
 * where w_n = exp(sign 2 pi i / n). Y_r are computed recursively. work must
 * hold 2n values.
 */
static void fft_rec(int n, int sign, const cplx *x, long s, cplx *y, cplx *work)
{
    if (n == 1) { y[0] = x[0]; return; }
    int p = smallest_factor(n);
    if (p == n) { oracle_dft1d(n, sign, x, s, y); return; }
    int m = n / p;
    cplx *sub = work;          /* p blocks of m values */
    cplx *rest = work + n;     /* scratch for the recursion */
    for (int r = 0; r < p; ++r)
        fft_rec(m, sign, x + (long)r * s, (long)p * s, sub + (long)r * m, rest);
    for (int u = 0; u < p; ++u)
        for (int q = 0; q < m; ++q) {
            int k = q + m * u;
            cplx acc = 0.0;
            for (int r = 0; r < p; ++r)
                acc += root_of_unity((long)r * k, n, sign) * sub[(long)r * m + q];
            y[k] = acc;
        }
}

/* Work space needed by fft_rec for length n: n + n/p + n/(p p') + ... <= 2n. */
void oracle_fft1d(int n, int sign, const cplx *x, long s, cplx *y)
{
    cplx *work = (cplx *)malloc(sizeof(cplx) * 2 * (size_t)n + sizeof(cplx));
    fft_rec(n, sign, x, s, y, work);
    free(work);
}

/* In-place 3-D transform of a C-ordered [n1][n2][n3] grid, one axis at a time. */
static void fft3d_inplace(const int *nn, int sign, cplx *g, cplx *line, cplx *out, cplx *work)
{
    const long n1 = nn[0], n2 = nn[1], n3 = nn[2];
    /* axis 3 (contiguous) */
    for (long a = 0; a < n1 * n2; ++a) {
        fft_rec((int)n3, sign, g + a * n3, 1, out, work);
        memcpy(g + a * n3, out, sizeof(cplx) * n3);
    }
    /* axis 2 */
    for (long i1 = 0; i1 < n1; ++i1)
        for (long i3 = 0; i3 < n3; ++i3) {
            cplx *base = g + i1 * n2 * n3 + i3;
            fft_rec((int)n2, sign, base, n3, out, work);
            for (long i2 = 0; i2 < n2; ++i2) base[i2 * n3] = out[i2];
        }
    /* axis 1 */
    for (long i2 = 0; i2 < n2; ++i2)
        for (long i3 = 0; i3 < n3; ++i3) {
            cplx *base = g + i2 * n3 + i3;
            fft_rec((int)n1, sign, base, n2 * n3, out, work);
            for (long i1 = 0; i1 < n1; ++i1) base[i1 * n2 * n3] = out[i1];
        }
    (void)line;
}

static long maxdim(const int *nn)
{
    long m = nn[0];
    if (nn[1] > m) m = nn[1];
    if (nn[2] > m) m = nn[2];
    return m;
}

/* 3-D transform of a [n1][n2][n3] grid: sign +1 = inverse (r from G), -1 = forward. */
void oracle_fft3d(const int *nn, int sign, cplx *g)
{
    long m = maxdim(nn);
    cplx *out = (cplx *)malloc(sizeof(cplx) * (size_t)m);
    cplx *work = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * m + 1));
    fft3d_inplace(nn, sign, g, NULL, out, work);
    free(out);
    free(work);
}

/* ---------------------------------------------------------------------- */
/* Geometry: reciprocal vectors, |k+G|^2, grid index of a Miller triple.   */
/* ---------------------------------------------------------------------- */

/* b_i with a_i . b_j = 2 pi delta_ij; lattice rows are a1, a2, a3. */
static void reciprocal_vectors(const double *a, double *b)
{
    const double *a1 = a, *a2 = a + 3, *a3 = a + 6;
    double c23[3] = {a2[1] * a3[2] - a2[2] * a3[1], a2[2] * a3[0] - a2[0] * a3[2], a2[0] * a3[1] - a2[1] * a3[0]};
    double c31[3] = {a3[1] * a1[2] - a3[2] * a1[1], a3[2] * a1[0] - a3[0] * a1[2], a3[0] * a1[1] - a3[1] * a1[0]};
    double c12[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2], a1[0] * a2[1] - a1[1] * a2[0]};
    double vol = a1[0] * c23[0] + a1[1] * c23[1] + a1[2] * c23[2];
    for (int c = 0; c < 3; ++c) {
        b[0 + c] = TWO_PI * c23[c] / vol;
        b[3 + c] = TWO_PI * c31[c] / vol;
        b[6 + c] = TWO_PI * c12[c] / vol;
    }
}

static double kplusg2(const double *b, const double *k, const int *m)
{
    double q[3];
    for (int c = 0; c < 3; ++c)
        q[c] = k[c] + m[0] * b[0 + c] + m[1] * b[3 + c] + m[2] * b[6 + c];
    return q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
}

static long wrap(int m, int n)
{
    int r = m % n;
    return r < 0 ? r + n : r;
}

static long grid_index(const int *nn, const int *m)
{
    return (wrap(m[0], nn[0]) * nn[1] + wrap(m[1], nn[1])) * (long)nn[2] + wrap(m[2], nn[2]);
}

/* ---------------------------------------------------------------------- */
/* The problem, as plain arrays (all host memory).                         */
/* ---------------------------------------------------------------------- */

typedef struct {
    double lattice[9];
    int fft[3];
    int nk;
    const double *kpts;      /* [nk][3] */
    const int *npw;          /* [nk] */
    const int *miller;       /* [sum npw][3] */
    const double *vloc;      /* [n1][n2][n3] */
    int nproj;
    int natom;
    const int *proj_atom_offset;   /* [natom+1] */
    const cplx *beta;        /* per k: [nproj][npw_k] */
    const double *dmat;      /* per atom: [np_a][np_a] row-major */
} oracle_problem;

static long pw_offset(const oracle_problem *p, int k)
{
    long o = 0;
    for (int i = 0; i < k; ++i) o += p->npw[i];
    return o;
}

/* Q = D P per atom block, for one band: q[i] = sum_j D_a[i][j] p[j]. */
static void apply_d(const oracle_problem *p, const cplx *proj, cplx *q)
{
    long doff = 0;
    for (int a = 0; a < p->natom; ++a) {
        int lo = p->proj_atom_offset[a], na = p->proj_atom_offset[a + 1] - lo;
        for (int i = 0; i < na; ++i) {
            cplx acc = 0.0;
            for (int j = 0; j < na; ++j) acc += p->dmat[doff + (long)i * na + j] * proj[lo + j];
            q[lo + i] = acc;
        }
        doff += (long)na * na;
    }
}

/*
 * y = H psi for nb bands at every k-point. psi, y: per k a [nb][npw_k] block.
 * terms: bit 0 kinetic, bit 1 local, bit 2 nonlocal (7 = full H).
 */
void oracle_apply_h(const oracle_problem *p, int nb, const cplx *psi, cplx *y, int terms)
{
    double b[9];
    reciprocal_vectors(p->lattice, b);
    const long N = (long)p->fft[0] * p->fft[1] * p->fft[2];
    for (int k = 0; k < p->nk; ++k) {
        const long off = pw_offset(p, k);
        const int npw = p->npw[k];
        const int *mil = p->miller + 3 * off;
        const cplx *bk = p->beta + (long)p->nproj * off;
        const cplx *pk = psi + (long)nb * off;
        cplx *yk = y + (long)nb * off;
        #pragma omp parallel
        {
            long m = maxdim(p->fft);
            cplx *grid = (cplx *)malloc(sizeof(cplx) * (size_t)N);
            cplx *out = (cplx *)malloc(sizeof(cplx) * (size_t)m);
            cplx *work = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * m + 1));
            cplx *proj = (cplx *)malloc(sizeof(cplx) * (size_t)(p->nproj + 1));
            cplx *q = (cplx *)malloc(sizeof(cplx) * (size_t)(p->nproj + 1));
            #pragma omp for schedule(static)
            for (int n = 0; n < nb; ++n) {
                const cplx *x = pk + (long)n * npw;
                cplx *r = yk + (long)n * npw;
                for (int g = 0; g < npw; ++g) r[g] = 0.0;
                if (terms & 1)
                    for (int g = 0; g < npw; ++g) r[g] += kplusg2(b, p->kpts + 3 * k, mil + 3 * g) * x[g];
                if (terms & 2) {
                    memset(grid, 0, sizeof(cplx) * (size_t)N);
                    for (int g = 0; g < npw; ++g) grid[grid_index(p->fft, mil + 3 * g)] = x[g];
                    fft3d_inplace(p->fft, +1, grid, NULL, out, work);
                    for (long j = 0; j < N; ++j) grid[j] *= p->vloc[j];
                    fft3d_inplace(p->fft, -1, grid, NULL, out, work);
                    for (int g = 0; g < npw; ++g) r[g] += grid[grid_index(p->fft, mil + 3 * g)] / (double)N;
                }
                if ((terms & 4) && p->nproj > 0) {
                    for (int i = 0; i < p->nproj; ++i) {
                        cplx acc = 0.0;
                        for (int g = 0; g < npw; ++g) acc += conj(bk[(long)i * npw + g]) * x[g];
                        proj[i] = acc;
                    }
                    apply_d(p, proj, q);
                    for (int g = 0; g < npw; ++g) {
                        cplx acc = 0.0;
                        for (int i = 0; i < p->nproj; ++i) acc += bk[(long)i * npw + g] * q[i];
                        r[g] += acc;
                    }
                }
            }
            free(grid); free(out); free(work); free(proj); free(q);
        }
    }
}

/* |k+G|^2 for every sphere point of k-point k (length npw[k]). */
void oracle_kinetic(const oracle_problem *p, int k, double *out)
{
    double b[9];
    reciprocal_vectors(p->lattice, b);
    const long off = pw_offset(p, k);
    for (int g = 0; g < p->npw[k]; ++g) out[g] = kplusg2(b, p->kpts + 3 * k, p->miller + 3 * (off + g));
}

/*
 * Explicit H matrix at k-point k, row-major [npw][npw], built from the
 * definition with no transform of psi:
 *   H[G][G'] = |k+G|^2 delta + Vt((m - m') mod N) + sum_ij beta_i(G) D_ij conj(beta_j(G'))
 *   Vt(q) = (1/N) sum_j V(r_j) exp(-2 pi i sum_l q_l j_l / N_l).
 * direct != 0 evaluates Vt by the O(N^2) sum (small grids only); otherwise by
 * the oracle's forward transform.
 */
void oracle_dense_h(const oracle_problem *p, int k, int direct, cplx *h)
{
    double b[9];
    reciprocal_vectors(p->lattice, b);
    const int n1 = p->fft[0], n2 = p->fft[1], n3 = p->fft[2];
    const long N = (long)n1 * n2 * n3;
    cplx *vt = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    if (direct) {
        #pragma omp parallel for schedule(static)
        for (long qi = 0; qi < N; ++qi) {
            long q1 = qi / ((long)n2 * n3), q2 = (qi / n3) % n2, q3 = qi % n3;
            cplx acc = 0.0;
            for (long j1 = 0; j1 < n1; ++j1)
                for (long j2 = 0; j2 < n2; ++j2)
                    for (long j3 = 0; j3 < n3; ++j3) {
                        double ph = TWO_PI * ((double)((q1 * j1) % n1) / n1 + (double)((q2 * j2) % n2) / n2 +
                                              (double)((q3 * j3) % n3) / n3);
                        acc += p->vloc[(j1 * n2 + j2) * n3 + j3] * (cos(ph) - I * sin(ph));
                    }
            vt[qi] = acc / (double)N;
        }
    } else {
        for (long j = 0; j < N; ++j) vt[j] = p->vloc[j];
        oracle_fft3d(p->fft, -1, vt);
        for (long j = 0; j < N; ++j) vt[j] /= (double)N;
    }
    const long off = pw_offset(p, k);
    const int npw = p->npw[k];
    const int *mil = p->miller + 3 * off;
    const cplx *bk = p->beta + (long)p->nproj * off;
    cplx *db = (cplx *)malloc(sizeof(cplx) * (size_t)p->nproj * (size_t)npw + 1);
    /* db[i][G'] = sum_j D_ij conj(beta_j(G')) */
    long doff = 0;
    for (int a = 0; a < p->natom; ++a) {
        int lo = p->proj_atom_offset[a], na = p->proj_atom_offset[a + 1] - lo;
        for (int i = 0; i < na; ++i)
            for (int g = 0; g < npw; ++g) {
                cplx acc = 0.0;
                for (int j = 0; j < na; ++j) acc += p->dmat[doff + (long)i * na + j] * conj(bk[(long)(lo + j) * npw + g]);
                db[(long)(lo + i) * npw + g] = acc;
            }
        doff += (long)na * na;
    }
    #pragma omp parallel for schedule(static)
    for (int g = 0; g < npw; ++g) {
        for (int gp = 0; gp < npw; ++gp) {
            int dm[3] = {mil[3 * g] - mil[3 * gp], mil[3 * g + 1] - mil[3 * gp + 1], mil[3 * g + 2] - mil[3 * gp + 2]};
            cplx v = vt[grid_index(p->fft, dm)];
            for (int i = 0; i < p->nproj; ++i) v += bk[(long)i * npw + g] * db[(long)i * npw + gp];
            if (g == gp) v += kplusg2(b, p->kpts + 3 * k, mil + 3 * g);
            h[(long)g * npw + gp] = v;
        }
    }
    free(db);
    free(vt);
}

/*
 * Adjoint of y = H psi for a real loss L with upstream g = dL/dRe y + i dL/dIm y:
 *   grad_psi = H g                       (H is Hermitian)
 *   grad_v(r_j) = (1/N) sum_{k,n} Re( conj(gamma_n(r_j)) psi_n(r_j) ),
 *       gamma_n, psi_n the unnormalised inverse transforms of g_n and psi_n
 *   grad_d[a](i,j) = Re sum_{k,n} Q_in conj(P_jn),  P = B^H psi, Q = B^H g
 * Any output pointer may be NULL. grad_v and grad_d are overwritten.
 */
void oracle_apply_h_backward(const oracle_problem *p, int nb, const cplx *psi, const cplx *dy,
                             cplx *grad_psi, double *grad_v, double *grad_d)
{
    if (grad_psi) oracle_apply_h(p, nb, dy, grad_psi, 7);
    const long N = (long)p->fft[0] * p->fft[1] * p->fft[2];
    long dlen = 0;
    for (int a = 0; a < p->natom; ++a) {
        long na = p->proj_atom_offset[a + 1] - p->proj_atom_offset[a];
        dlen += na * na;
    }
    if (grad_v) memset(grad_v, 0, sizeof(double) * (size_t)N);
    if (grad_d) memset(grad_d, 0, sizeof(double) * (size_t)dlen);
    const int nthr = omp_get_max_threads();
    double *gv_part = grad_v ? (double *)calloc((size_t)N * (size_t)nthr, sizeof(double)) : NULL;
    double *gd_part = grad_d ? (double *)calloc((size_t)(dlen + 1) * (size_t)nthr, sizeof(double)) : NULL;
    for (int k = 0; k < p->nk; ++k) {
        const long off = pw_offset(p, k);
        const int npw = p->npw[k];
        const int *mil = p->miller + 3 * off;
        const cplx *bk = p->beta + (long)p->nproj * off;
        #pragma omp parallel
        {
            const int t = omp_get_thread_num();
            long m = maxdim(p->fft);
            cplx *ga = (cplx *)malloc(sizeof(cplx) * (size_t)N);
            cplx *gb = (cplx *)malloc(sizeof(cplx) * (size_t)N);
            cplx *out = (cplx *)malloc(sizeof(cplx) * (size_t)m);
            cplx *work = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * m + 1));
            cplx *pp = (cplx *)malloc(sizeof(cplx) * (size_t)(p->nproj + 1));
            cplx *qq = (cplx *)malloc(sizeof(cplx) * (size_t)(p->nproj + 1));
            #pragma omp for schedule(static)
            for (int n = 0; n < nb; ++n) {
                const cplx *x = psi + (long)nb * off + (long)n * npw;
                const cplx *gy = dy + (long)nb * off + (long)n * npw;
                if (grad_v) {
                    memset(ga, 0, sizeof(cplx) * (size_t)N);
                    memset(gb, 0, sizeof(cplx) * (size_t)N);
                    for (int g = 0; g < npw; ++g) {
                        long idx = grid_index(p->fft, mil + 3 * g);
                        ga[idx] = x[g];
                        gb[idx] = gy[g];
                    }
                    fft3d_inplace(p->fft, +1, ga, NULL, out, work);
                    fft3d_inplace(p->fft, +1, gb, NULL, out, work);
                    double *acc = gv_part + (long)t * N;
                    for (long j = 0; j < N; ++j) acc[j] += creal(conj(gb[j]) * ga[j]) / (double)N;
                }
                if (grad_d && p->nproj > 0) {
                    for (int i = 0; i < p->nproj; ++i) {
                        cplx a1 = 0.0, a2 = 0.0;
                        for (int g = 0; g < npw; ++g) {
                            a1 += conj(bk[(long)i * npw + g]) * x[g];
                            a2 += conj(bk[(long)i * npw + g]) * gy[g];
                        }
                        pp[i] = a1;
                        qq[i] = a2;
                    }
                    double *acc = gd_part + (long)t * (dlen + 1);
                    long doff = 0;
                    for (int a = 0; a < p->natom; ++a) {
                        int lo = p->proj_atom_offset[a], na = p->proj_atom_offset[a + 1] - lo;
                        for (int i = 0; i < na; ++i)
                            for (int j = 0; j < na; ++j)
                                acc[doff + (long)i * na + j] += creal(qq[lo + i] * conj(pp[lo + j]));
                        doff += (long)na * na;
                    }
                }
            }
            free(ga); free(gb); free(out); free(work); free(pp); free(qq);
        }
    }
    for (int t = 0; t < nthr; ++t) {
        if (grad_v)
            for (long j = 0; j < N; ++j) grad_v[j] += gv_part[(long)t * N + j];
        if (grad_d)
            for (long j = 0; j < dlen; ++j) grad_d[j] += gd_part[(long)t * (dlen + 1) + j];
    }
    free(gv_part);
    free(gd_part);
}

/*
 * Electron density on the grid: the k-weighted sum over orbitals of the squared
 * modulus of each orbital's real-space values, as in the plane-wave density of
 * Sec. III.C (the e^{ik.r} factor has modulus one and drops out), written with
 * the unnormalised transform of the coefficients (no 1/Omega):
 *   rho(r_j) = sum_{k,n} occ[k][n] |psi_nk(r_j)|^2,
 *   psi_nk(r_j) = sum_{G in S_k} c_nk(G) exp(+i G.r_j)   (inverse transform of the
 *   coefficients scattered to the grid, Miller index m -> m mod N).
 * occ holds the weight of each band (k-point weight times occupation).
 * rho is overwritten.
 */
void oracle_density(const oracle_problem *p, int nb, const cplx *psi, const double *occ, double *rho)
{
    const long N = (long)p->fft[0] * p->fft[1] * p->fft[2];
    const int nthr = omp_get_max_threads();
    double *part = (double *)calloc((size_t)N * (size_t)nthr, sizeof(double));
    for (int k = 0; k < p->nk; ++k) {
        const long off = pw_offset(p, k);
        const int npw = p->npw[k];
        const int *mil = p->miller + 3 * off;
        #pragma omp parallel
        {
            const int t = omp_get_thread_num();
            long m = maxdim(p->fft);
            cplx *ga = (cplx *)malloc(sizeof(cplx) * (size_t)N);
            cplx *out = (cplx *)malloc(sizeof(cplx) * (size_t)m);
            cplx *work = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * m + 1));
            #pragma omp for schedule(static)
            for (int n = 0; n < nb; ++n) {
                const cplx *x = psi + (long)nb * off + (long)n * npw;
                const double w = occ[(long)k * nb + n];
                memset(ga, 0, sizeof(cplx) * (size_t)N);
                for (int g = 0; g < npw; ++g) ga[grid_index(p->fft, mil + 3 * g)] = x[g];
                fft3d_inplace(p->fft, +1, ga, NULL, out, work);
                double *acc = part + (long)t * N;
                for (long j = 0; j < N; ++j) acc[j] += w * (creal(ga[j]) * creal(ga[j]) + cimag(ga[j]) * cimag(ga[j]));
            }
            free(ga); free(out); free(work);
        }
    }
    memset(rho, 0, sizeof(double) * (size_t)N);
    for (int t = 0; t < nthr; ++t)
        for (long j = 0; j < N; ++j) rho[j] += part[(long)t * N + j];
    free(part);
}

int oracle_num_threads(void) { return omp_get_max_threads(); }

/* Sets the OpenMP thread count of later calls (the CPU baseline times 1 thread and all threads). */
void oracle_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

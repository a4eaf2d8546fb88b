// Nonlocal (Kleinman-Bylander) force on the atoms (abacus_pw_force_nl).
//
// Sec. III.A gives the nonlocal force as the derivative of the projector
// energy with respect to the atomic positions. The projectors of atom a carry
// the structure factor exp(-i (k+G).tau_a), so d beta / d tau_alpha =
// -i (k+G)_alpha beta, and with E_NL = sum_k sum_n occ[k][n] sum_a P_a^H D_a P_a:
//   F[a][alpha] = -dE_NL/dtau_{a,alpha}
//               = -2 sum_k sum_n occ[k][n] sum_{i,j in a} D_ij Im(conj(P^alpha_in) P_jn),
//   P = B^H psi,  P^alpha = B^H ((k+G)_alpha psi).
// Per k-point the four projections come from one GEMM against the stacked
// operator [B; (k+G)_x B; (k+G)_y B; (k+G)_z B] (4 nproj rows, formed by one
// pass over beta), then one work-group per atom reduces over bands in a fixed
// order and adds the k-point's share to F (k-points in order).
#include <algorithm>

#include "gemm.hpp"
#include "hamiltonian.hpp"

namespace apw {

namespace {

constexpr int kMaxAtomProj = 16;   // projectors per atom handled by the reduction

// out[r nproj + i][g] = (r == 0 ? 1 : kg[g][r - 1]) beta[i][g]
__global__ __launch_bounds__(256) void k_force_stack(int nproj, int npw, const z64 *__restrict__ beta,
                                                     const double *__restrict__ kg, z64 *__restrict__ out) {
    const int64_t n = (int64_t)nproj * npw;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const int g = (int)(e % npw);
        const z64 b = beta[e];
        const double gx = kg[3 * (int64_t)g], gy = kg[3 * (int64_t)g + 1], gz = kg[3 * (int64_t)g + 2];
        out[e] = b;
        out[n + e] = b * gx;
        out[2 * n + e] = b * gy;
        out[3 * n + e] = b * gz;
    }
}

// One work-group per atom: acc_alpha = sum_n occ[n] sum_{i,j} D_ij Im(conj(Pa_in) P_jn) with
// Pall column-major [nb][4 nproj] (P rows 0..nproj-1, then P^x, P^y, P^z);
// force[a][alpha] (=, or += when accumulate) -2 acc_alpha.
__global__ __launch_bounds__(256) void k_force_reduce(int nb, int nproj, const z64 *__restrict__ pall,
                                                      const double *__restrict__ occ, const int *__restrict__ aoff,
                                                      const double *__restrict__ dmat, double *__restrict__ force,
                                                      int accumulate) {
    const int a = blockIdx.x;
    const int lo = aoff[a], na = aoff[a + 1] - lo;
    // the atom's D block starts after the blocks of the atoms before it
    int64_t doff = 0;
    for (int b = 0; b < a; ++b) {
        const int nb2 = aoff[b + 1] - aoff[b];
        doff += (int64_t)nb2 * nb2;
    }
    __shared__ double dsh[kMaxAtomProj * kMaxAtomProj];
    __shared__ double red[3][256];
    for (int q = threadIdx.x; q < na * na; q += blockDim.x) dsh[q] = dmat[doff + q];
    __syncthreads();
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t ld = 4 * (int64_t)nproj;
    for (int n = threadIdx.x; n < nb; n += blockDim.x) {
        const z64 *col = pall + (int64_t)n * ld;
        double s[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < na; ++i) {
            z64 q{0.0, 0.0};
            for (int j = 0; j < na; ++j) q = q + col[lo + j] * dsh[i * na + j];
            for (int al = 0; al < 3; ++al) {
                const z64 pa = col[(int64_t)(al + 1) * nproj + lo + i];
                s[al] += pa.re * q.im - pa.im * q.re;   // Im(conj(pa) q)
            }
        }
        const double w = occ[n];
        for (int al = 0; al < 3; ++al) acc[al] += w * s[al];
    }
    for (int al = 0; al < 3; ++al) red[al][threadIdx.x] = acc[al];
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int al = 0; al < 3; ++al) red[al][threadIdx.x] += red[al][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        const double v = -2.0 * red[threadIdx.x][0];
        double *o = force + 3 * (int64_t)a + threadIdx.x;
        *o = accumulate ? *o + v : v;
    }
}

__global__ void k_force_zero(int n, double *__restrict__ f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) f[i] = 0.0;
}

int force_tables(const abacus_pw_problem &p, Plan &P, hipStream_t st) {
    if (P.force_tab_ready) return ABACUS_PW_OK;
    std::vector<double> kg(3 * (size_t)P.npw_total);
    for (int k = 0; k < P.nk; ++k) {
        const int *mk = p.miller + 3 * P.pw_off[k];
        const double *kv = p.kpts + 3 * k;
        for (int g = 0; g < P.npw[k]; ++g) {
            const int *m = mk + 3 * g;
            double *o = kg.data() + 3 * (size_t)(P.pw_off[k] + g);
            for (int c = 0; c < 3; ++c) o[c] = kv[c] + m[0] * P.recip[c] + m[1] * P.recip[3 + c] + m[2] * P.recip[6 + c];
        }
    }
    const size_t kb = sizeof(double) * kg.size(), ab = sizeof(int) * P.proj_atom_offset.size();
    APW_TRY(P.force_tab.ensure(kb + ab));
    APW_HIP(hipMemcpyAsync(P.force_tab.ptr, kg.data(), kb, hipMemcpyHostToDevice, st));
    APW_HIP(hipMemcpyAsync(P.force_tab.as<char>() + kb, P.proj_atom_offset.data(), ab, hipMemcpyHostToDevice, st));
    APW_HIP(hipStreamSynchronize(st));   // the host vectors go out of scope
    P.force_tab_ready = true;
    return ABACUS_PW_OK;
}

}  // namespace

int force_nl_all(const abacus_pw_problem &p, Plan &P, int nb, const void *psi, const double *occ, double *force,
                 hipStream_t st) {
    if (P.natom == 0) return ABACUS_PW_OK;
    if (P.nproj == 0) {   // no projectors: no nonlocal force
        hipLaunchKernelGGL(k_force_zero, dim3(ceil_div(3 * P.natom, 256)), dim3(256), 0, st, 3 * P.natom, force);
        return check_launch("force_zero");
    }
    for (int a = 0; a < P.natom; ++a)
        if (P.proj_atom_offset[a + 1] - P.proj_atom_offset[a] > kMaxAtomProj)
            return set_error(ABACUS_PW_EBAD_SHAPE, "more than 16 projectors on one atom");
    APW_TRY(force_tables(p, P, st));
    const double *kg_all = P.force_tab.as<double>();
    const int *aoff = reinterpret_cast<const int *>(P.force_tab.as<char>() + sizeof(double) * 3 * (size_t)P.npw_total);
    const int m4 = 4 * P.nproj;
    APW_TRY(P.force_stack.ensure(sizeof(z64) * (size_t)m4 * P.max_npw));
    APW_TRY(P.proj.ensure(sizeof(z64) * (size_t)m4 * nb));
    APW_TRY(P.gemm_part.ensure(gemm_cn_part_bytes(m4, nb, P.max_npw, 16, g_splitk_chunk)));
    for (int k = 0; k < P.nk; ++k) {
        const KTables &K = P.k[k];
        const z64 *bk = static_cast<const z64 *>(p.beta) + (size_t)P.nproj * K.pw_off;
        const z64 *xk = static_cast<const z64 *>(psi) + (size_t)nb * K.pw_off;
        {
            KernelTimer kt("force_stack", st);
            const int64_t n = (int64_t)P.nproj * K.npw;
            hipLaunchKernelGGL(k_force_stack, dim3((unsigned)std::min<int64_t>(ceil_div64(n, 256), 8192)), dim3(256),
                               0, st, P.nproj, K.npw, bk, kg_all + 3 * K.pw_off, P.force_stack.as<z64>());
            APW_TRY(check_launch("force_stack"));
        }
        APW_TRY(gemm_cn(0, m4, nb, K.npw, P.force_stack.ptr, K.npw, xk, K.npw, P.proj.ptr, m4, 1.0, 0.0,
                        P.gemm_part.ptr, g_splitk_chunk, st));
        KernelTimer kt("force_reduce", st);
        hipLaunchKernelGGL(k_force_reduce, dim3(P.natom), dim3(256), 0, st, nb, P.nproj, P.proj.as<z64>(),
                           occ + (size_t)k * nb, aoff, static_cast<const double *>(p.dmat), force, k > 0 ? 1 : 0);
        APW_TRY(check_launch("force_reduce"));
    }
    return ABACUS_PW_OK;
}

}  // namespace apw

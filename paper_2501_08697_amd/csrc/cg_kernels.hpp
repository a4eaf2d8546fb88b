// Kernels of the band-by-band conjugate-gradient eigensolver; see cg_kernels.hip.
#pragma once

#include "common.hpp"

namespace apw {

// Scalars of one band's CG iteration, kept in device memory so that a step
// needs no host round trip except for the convergence test.
struct CgScalars {
    double lam;           // Rayleigh quotient <psi|p>
    double rn2, ek;       // ||p - lam psi||^2, sum_G |k+G|^2 |psi|^2
    double gr, grp;       // Re<g|r>, Re<g|r_prev>
    double gr_prev;       // Re<g|r> of the previous step
    double dn2;           // ||d_perp||^2
    double b, c;          // Re<p|d_hat>, <d_hat|H d_hat>
    z64 xd;               // <psi|d>
    z64 a1, b1;           // coefficients of the pending linear combination
    z64 a2, b2;
};

// out = a * u + b * v for complex vectors of length n; a, b read from device memory.
int cg_axpby(int n, const z64 *a, const z64 *u, const z64 *b, const z64 *v, z64 *out, hipStream_t st);
// Complex inner products <u1|v1> and, if u2 is given, <u2|v2> (fixed summation order),
// written to out1 / out2 (re, im); only the real part when re_only.
int cg_dots(int n, const z64 *u1, const z64 *v1, double *out1, const z64 *u2, const z64 *v2, double *out2,
            bool re_only, hipStream_t st);
// Scalar stages (one thread each); see cg_kernels.hip.
int cg_stage_direction(CgScalars *s, int first, hipStream_t st);
int cg_stage_project(CgScalars *s, hipStream_t st);
int cg_stage_normalise(CgScalars *s, hipStream_t st);
int cg_stage_rotate(CgScalars *s, hipStream_t st);
int cg_stage_scale_self(CgScalars *s, hipStream_t st);
int cg_zero(int n, z64 *x, hipStream_t st);

}  // namespace apw

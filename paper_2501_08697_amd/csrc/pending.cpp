// Entry points whose drivers are not compiled in yet report EINTERNAL.
#include "hamiltonian.hpp"

namespace apw {

int apply_h_backward_all(const abacus_pw_problem &, Plan &, int, int, const void *, const void *, void *, double *,
                         double *, hipStream_t) {
    return set_error(ABACUS_PW_EINTERNAL, "adjoint not available in this build");
}

}  // namespace apw

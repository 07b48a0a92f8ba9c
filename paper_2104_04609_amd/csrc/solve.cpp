// GMRES solve (placeholder).
#include "bem_internal.h"

extern "C" {
void bem_solve_opts_default(bem_solve_opts *o) {
    o->pade_terms = 4;
    o->theta = M_PI / 3;
    o->osrc_interior = 1;
    o->R = 0;
    o->precision = BEM_FP64;
    o->maxiter = 1000;
    o->inner_tol = 1e-5;
    o->max_outer = 8;
}
int pmchwt_solve(const bem_mesh *, bem_c64, bem_c64, double, const double *, int, double,
                 const bem_solve_opts *, bem_c64 *, bem_solve_info *, void *) {
    return BEM_E_UNSUPPORTED;
}
}

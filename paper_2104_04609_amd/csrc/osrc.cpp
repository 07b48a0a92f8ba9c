// OSRC preconditioner (placeholder until the factorisation lands).
#include "bem_internal.h"

namespace bem {
struct OsrcState {};
void OsrcDeleter::operator()(OsrcState *p) const { delete p; }
int64_t osrc_bytes(const OsrcState &) { return 0; }
OsrcState &osrc_get(bem_mesh *, int, double, double2, const std::vector<double2> &,
                    hipStream_t) {
    fail(BEM_E_UNSUPPORTED, "OSRC not built yet");
}
void osrc_apply_strong(bem_mesh *, OsrcState &, const double2 *, double2 *, hipStream_t) {}
void osrc_apply_from_weak(bem_mesh *, OsrcState &, const double2 *, double2 *, hipStream_t) {}
void osrc_mass_solve(bem_mesh *, OsrcState &, const double2 *, double2 *, int, hipStream_t) {}
}   // namespace bem

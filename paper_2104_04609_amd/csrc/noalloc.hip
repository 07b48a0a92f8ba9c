// osrc_apply_noalloc: the OSRC preconditioner apply (Sec. 2.6, 2.7) for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).  The factors come from the
// mesh handle's cache (an earlier osrc_apply or pmchwt_solve with the same
// parameters created them); the per-vector work vectors of the level sweeps
// live in `scratch`, a device array of fixed size that every GPU the library
// runs on holds until the process ends.  Its device address is taken once per
// device with hipGetSymbolAddress: in host code the array's name is only a
// host-side stand-in.
#include <map>
#include <mutex>

#include "osrc_internal.h"

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;   // BEM_NOALLOC_SCRATCH_BYTES
static_assert(NOALLOC_SCRATCH_BYTES == BEM_NOALLOC_SCRATCH_BYTES, "header and library disagree");

static __device__ __align__(256) double2 scratch[NOALLOC_SCRATCH_BYTES / sizeof(double2)];

std::mutex g_scratch_mu;
std::map<int, double2 *> g_scratch_ptr;   // device ordinal -> address of scratch there

// Address of this device's copy of scratch (current device), looked up on the
// first call on each device.
double2 *scratch_ptr() {
    int dev = -1;
    BEM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) return it->second;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        bem::fail(BEM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double2 *>(p);
    return static_cast<double2 *>(p);
}

}   // namespace

extern "C" int osrc_apply_noalloc(const bem_mesh *mesh, int pade_terms, double theta, bem_c64 k,
                                  bem_c64 k_eps, const bem_c64 *x, bem_c64 *y, int n_rhs,
                                  void *hip_stream) {
    try {
        if (!mesh) bem::fail(BEM_E_INVAL, "mesh is NULL");
        if (pade_terms < 1 || pade_terms > bem::PADE_MAX)
            bem::fail(BEM_E_INVAL, "pade_terms must be in 1..32");
        if (!std::isfinite(theta)) bem::fail(BEM_E_INVAL, "theta not finite");
        if (!std::isfinite(k.re) || !std::isfinite(k.im) || (k.re == 0 && k.im == 0))
            bem::fail(BEM_E_INVAL, "k must be finite and nonzero");
        if (!std::isfinite(k_eps.re) || !std::isfinite(k_eps.im) ||
            (k_eps.re == 0 && k_eps.im == 0))
            bem::fail(BEM_E_INVAL, "k_eps must be finite and nonzero");
        if (!x || !y || x == y) bem::fail(BEM_E_INVAL, "x, y must be distinct device pointers");
        if (n_rhs < 1) bem::fail(BEM_E_INVAL, "n_rhs must be >= 1");
        bem_mesh *m = const_cast<bem_mesh *>(mesh);
        const std::vector<double2> keps(m->nobj, make_double2(k_eps.re, k_eps.im));
        bem::OsrcState *st =
            bem::osrc_find(m, pade_terms, theta, make_double2(k.re, k.im), keps);
        if (!st)
            bem::fail(BEM_E_INVAL, "no OSRC factors for these parameters on this mesh handle: "
                                   "call osrc_apply (or pmchwt_solve) with them once first");
        const int64_t n = m->N, n2 = 2 * n;
        const int batch = std::min(n_rhs, 16);   // right-hand sides per pass, as osrc_apply
        const int64_t per = bem::osrc_scratch_per_rhs(m, pade_terms);
        const int64_t cap = (int64_t)(NOALLOC_SCRATCH_BYTES / sizeof(double2));
        if ((int64_t)batch * per > cap)
            bem::fail(BEM_E_INVAL,
                      "the work vectors of min(n_rhs, 16) right-hand sides need " +
                          std::to_string((int64_t)batch * per * 16) +
                          " bytes, which exceeds the no-allocation scratch of " +
                          std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes");
        const bem::OsrcScratch scr = bem::osrc_scratch_at(m, pade_terms, batch, scratch_ptr());
        const bem::NoTimerScope no_events;
        hipStream_t s = (hipStream_t)hip_stream;
        for (int r0 = 0; r0 < n_rhs; r0 += batch)
            bem::osrc_apply_strong(m, *st, (const double2 *)x + r0 * n2, (double2 *)y + r0 * n2,
                                   std::min(batch, n_rhs - r0), s, &scr);
        return BEM_OK;
    } catch (const bem::Error &e) {
        bem::set_last_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        bem::set_last_error(e.what());
        return BEM_E_DEVICE;
    }
}

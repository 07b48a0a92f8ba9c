// C ABI entry points: argument validation, error reporting, kernel timing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "bem_internal.h"

namespace bem {

namespace {
thread_local std::string g_last_error;

struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;

void prof_clear_locked() {
    for (auto &r : g_prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.clear();
}
}   // namespace

[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }

void set_last_error(const std::string &msg) { g_last_error = msg; }

namespace {
std::mutex g_rel_mu;
std::vector<std::pair<MemReleaser, void *>> g_releasers;
}   // namespace

void add_mem_releaser(MemReleaser fn, void *ctx) {
    std::lock_guard<std::mutex> g(g_rel_mu);
    g_releasers.emplace_back(fn, ctx);
}
void remove_mem_releaser(void *ctx) {
    std::lock_guard<std::mutex> g(g_rel_mu);
    g_releasers.erase(std::remove_if(g_releasers.begin(), g_releasers.end(),
                                     [&](const std::pair<MemReleaser, void *> &r) {
                                         return r.second == ctx;
                                     }),
                      g_releasers.end());
}
bool release_device_memory() {
    std::vector<std::pair<MemReleaser, void *>> rs;
    {
        std::lock_guard<std::mutex> g(g_rel_mu);
        rs = g_releasers;
    }
    for (const auto &r : rs)
        if (r.first(r.second)) return true;
    return false;
}

namespace {
thread_local bool t_no_timer = false;
}

NoTimerScope::NoTimerScope() : prev(t_no_timer) { t_no_timer = true; }
NoTimerScope::~NoTimerScope() { t_no_timer = prev; }

Timer::Timer(const char *kernel, hipStream_t stream) : name(kernel), s(stream) {
    if (t_no_timer) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (!g_prof_on) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        a = b = nullptr;
        return;
    }
    (void)hipEventRecord(a, s);
}

Timer::~Timer() {
    if (!a) return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof.push_back({name, a, b});
}

}   // namespace bem

bem_mesh::~bem_mesh() = default;

namespace bem {
Tuning &tuning() {
    static Tuning t;
    return t;
}

void mesh_trim(bem_mesh *m) {
    m->near_cache.clear();
    m->dense_cache.clear();
    m->dense64_cache.clear();
    m->dense_rounded_cache.clear();
    m->hmat_cache.clear();
    m->osrc_cache.clear();
    m->xs32.release();
    m->dyn64.release();
    m->dyn32.release();
    m->partial.release();
    m->trirows.release();
    m->sym_items.release();
    m->sym_plan_id = nullptr;
    m->parts.clear();
    m->part_vidx.clear();
}
}   // namespace bem

int64_t bem_mesh::device_bytes() const {
    int64_t b = geo64.bytes() + geo32.bytes() + tst.bytes() + tobj_d.bytes() + tri_d.bytes() +
                star_ptr.bytes() + star_idx.bytes() + near_pairs.bytes() + nf_rowptr.bytes() +
                nf_col.bytes() + nf_cptr.bytes() + nf_contrib.bytes() + ss_tab.bytes() +
                dyn64.bytes() + dyn32.bytes() + partial.bytes() + trirows.bytes() +
                sym_items.bytes() + P_d.bytes();
    for (const auto &kv : near_cache) b += kv.second->vals.bytes();
    for (const auto &kv : dense_cache) b += kv.second->bytes();
    for (const auto &kv : dense64_cache) b += kv.second->bytes();
    for (const auto &kv : dense_rounded_cache) b += kv.second->bytes();
    for (const auto &kv : hmat_cache) b += bem::hmat_bytes(*kv.second);
    b += xs32.bytes();
    for (const auto &kv : osrc_cache) b += bem::osrc_bytes(*kv.second);
    if (osrc_sym) b += bem::osrc_sym_bytes(*osrc_sym);
    for (const auto &pm : parts) b += pm->device_bytes();
    for (const auto &v : part_vidx) b += v.bytes();
    return b;
}

using bem::fail;

#define BEM_API_BEGIN try {
#define BEM_API_END                                                              \
    }                                                                            \
    catch (const bem::Error &e) {                                                \
        bem::g_last_error = e.msg;                                               \
        return e.code;                                                           \
    }                                                                            \
    catch (const std::bad_alloc &) {                                             \
        bem::g_last_error = "host allocation failed";                           \
        return BEM_E_NOMEM;                                                      \
    }                                                                            \
    catch (const std::exception &e) {                                            \
        bem::g_last_error = e.what();                                            \
        return BEM_E_DEVICE;                                                     \
    }

namespace {

void check_k(bem_c64 k, const char *name) {
    if (!std::isfinite(k.re) || !std::isfinite(k.im))
        fail(BEM_E_INVAL, std::string(name) + " is not finite");
    if (k.im < 0) fail(BEM_E_INVAL, std::string(name) + " must have Im k >= 0");
    if (k.re == 0 && k.im == 0) fail(BEM_E_INVAL, std::string(name) + " must be nonzero");
}

void check_mesh(const bem_mesh *m) {
    if (!m) fail(BEM_E_INVAL, "mesh is NULL");
}

}   // namespace

extern "C" {

const char *bem_last_error(void) { return bem::g_last_error.c_str(); }

int bem_mesh_create(const double *vertices, int64_t n_vertices, const int32_t *triangles,
                    int64_t n_triangles, const int32_t *object_id, bem_mesh **out) {
    BEM_API_BEGIN
    bem::g_last_error.clear();
    if (!out) fail(BEM_E_INVAL, "out is NULL");
    *out = nullptr;
    auto m = std::make_unique<bem_mesh>();
    bem::mesh_build(m.get(), vertices, n_vertices, triangles, n_triangles, object_id);
    *out = m.release();
    return BEM_OK;
    BEM_API_END
}

void bem_mesh_destroy(bem_mesh *mesh) { delete mesh; }

int bem_mesh_info(const bem_mesh *m, int64_t *nv, int64_t *nt, int32_t *nobj,
                  int64_t *bytes) {
    BEM_API_BEGIN
    check_mesh(m);
    if (nv) *nv = m->N;
    if (nt) *nt = m->T;
    if (nobj) *nobj = m->nobj;
    if (bytes) *bytes = m->device_bytes();
    return BEM_OK;
    BEM_API_END
}

}   // extern "C"

namespace {

// Per-object interior wavenumbers and density ratios, checked; throws.
bem::ObjMaterials materials(const bem_mesh *mesh, const bem_c64 *k_int, const double *rho) {
    if (!k_int || !rho) fail(BEM_E_INVAL, "k_int and rho must not be NULL");
    check_mesh(mesh);
    bem::ObjMaterials om;
    for (int o = 0; o < mesh->nobj; o++) {
        om.k.push_back(make_double2(k_int[o].re, k_int[o].im));
        om.rho.push_back(rho[o]);
    }
    bem::check_materials(mesh, om);
    return om;
}

// Body of pmchwt_matvec (s1 = +1) and muller_matvec (s1 = -1); throws.
void operator_matvec(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int, double rho,
                     const bem_c64 *x, bem_c64 *y, int n_rhs, int precision,
                     void *hip_stream, int s1, const bem::ObjMaterials *om = nullptr) {
    check_mesh(mesh);
    check_k(k_ext, "k_ext");
    check_k(k_int, "k_int");
    if (!(rho > 0) || !std::isfinite(rho)) fail(BEM_E_INVAL, "rho must be positive");
    if (!x || !y) fail(BEM_E_INVAL, "x and y must be device pointers");
    if (x == y) fail(BEM_E_INVAL, "x and y must not alias");
    if (n_rhs < 1) fail(BEM_E_INVAL, "n_rhs must be >= 1");
    if (precision != BEM_FP64 && precision != BEM_FP32 && precision != BEM_FP32_DENSE &&
        precision != BEM_FP64_DENSE && precision != BEM_FP32_HMAT)
        fail(BEM_E_INVAL, "bad precision");
    bem_mesh *m = const_cast<bem_mesh *>(mesh);
    hipStream_t s = (hipStream_t)hip_stream;
    double2 k0 = make_double2(k_ext.re, k_ext.im), k1 = make_double2(k_int.re, k_int.im);
    const bem::NearOperator &nf = bem::nearfield_get(m, k0, k1, rho, s, s1, om);
    if (precision == BEM_FP32_DENSE || precision == BEM_FP64_DENSE) {
        const bem::DenseOperator &op =
            bem::dense_get(m, k0, k1, rho, s, s1, om, precision == BEM_FP64_DENSE);
        bem::dense_apply(op, (const double2 *)x, (double2 *)y, n_rhs, m->xs32, s);
        return;
    }
    if (precision == BEM_FP32_HMAT) {
        bem::HMatrix &h = bem::hmat_get(m, k0, k1, rho, s, s1, om);
        const int64_t n2 = 2 * m->N;
        for (int r = 0; r < n_rhs; r++)
            bem::hmat_apply(h, m, nf, (const double2 *)x + r * n2, (double2 *)y + r * n2, s);
        return;
    }
    bem::farfield_apply_batch(m, nf, k0, k1, rho, (const double2 *)x, (double2 *)y, n_rhs,
                              precision, s);
}

}   // namespace

extern "C" {

int pmchwt_matvec(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int, double rho,
                  const bem_c64 *x, bem_c64 *y, int n_rhs, int precision,
                  void *hip_stream) {
    BEM_API_BEGIN
    operator_matvec(mesh, k_ext, k_int, rho, x, y, n_rhs, precision, hip_stream, 1);
    return BEM_OK;
    BEM_API_END
}

int pmchwt_matvec_multi(const bem_mesh *mesh, bem_c64 k_ext, const bem_c64 *k_int,
                        const double *rho, const bem_c64 *x, bem_c64 *y, int n_rhs,
                        int precision, void *hip_stream) {
    BEM_API_BEGIN
    const bem::ObjMaterials om = materials(mesh, k_int, rho);
    operator_matvec(mesh, k_ext, k_int[0], rho[0], x, y, n_rhs, precision, hip_stream, 1, &om);
    return BEM_OK;
    BEM_API_END
}

int muller_matvec(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int, double rho,
                  const bem_c64 *x, bem_c64 *y, int n_rhs, int precision,
                  void *hip_stream) {
    BEM_API_BEGIN
    operator_matvec(mesh, k_ext, k_int, rho, x, y, n_rhs, precision, hip_stream, -1);
    return BEM_OK;
    BEM_API_END
}

int osrc_apply(const bem_mesh *mesh, int pade_terms, double theta, bem_c64 k,
               bem_c64 k_eps, const bem_c64 *x, bem_c64 *y, int n_rhs, void *hip_stream) {
    BEM_API_BEGIN
    check_mesh(mesh);
    if (pade_terms < 1 || pade_terms > 32) fail(BEM_E_INVAL, "pade_terms must be in 1..32");
    if (!std::isfinite(theta)) fail(BEM_E_INVAL, "theta not finite");
    if (!std::isfinite(k.re) || !std::isfinite(k.im) || (k.re == 0 && k.im == 0))
        fail(BEM_E_INVAL, "k must be finite and nonzero");
    if (!std::isfinite(k_eps.re) || !std::isfinite(k_eps.im) ||
        (k_eps.re == 0 && k_eps.im == 0))
        fail(BEM_E_INVAL, "k_eps must be finite and nonzero");
    if (!x || !y || x == y) fail(BEM_E_INVAL, "x, y must be distinct device pointers");
    if (n_rhs < 1) fail(BEM_E_INVAL, "n_rhs must be >= 1");
    bem_mesh *m = const_cast<bem_mesh *>(mesh);
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<double2> keps(m->nobj, make_double2(k_eps.re, k_eps.im));
    bem::OsrcState &st =
        bem::osrc_get(m, pade_terms, theta, make_double2(k.re, k.im), keps, s);
    const int64_t n2 = 2 * m->N;
    for (int r0 = 0; r0 < n_rhs; r0 += 16)   // batches of up to 16 right-hand sides
        bem::osrc_apply_strong(m, st, (const double2 *)x + r0 * n2, (double2 *)y + r0 * n2,
                               std::min(16, n_rhs - r0), s);
    return BEM_OK;
    BEM_API_END
}

int bem_osrc_info(const bem_mesh *mesh, int pade_terms, double theta, bem_c64 k, bem_c64 k_eps,
                  bem_osrc_stats *out, void *hip_stream) {
    BEM_API_BEGIN
    check_mesh(mesh);
    if (pade_terms < 1 || pade_terms > 32) fail(BEM_E_INVAL, "pade_terms must be in 1..32");
    if (!std::isfinite(theta)) fail(BEM_E_INVAL, "theta not finite");
    if (!std::isfinite(k.re) || !std::isfinite(k.im) || (k.re == 0 && k.im == 0))
        fail(BEM_E_INVAL, "k must be finite and nonzero");
    if (!std::isfinite(k_eps.re) || !std::isfinite(k_eps.im) ||
        (k_eps.re == 0 && k_eps.im == 0))
        fail(BEM_E_INVAL, "k_eps must be finite and nonzero");
    if (!out) fail(BEM_E_INVAL, "out is NULL");
    bem_mesh *m = const_cast<bem_mesh *>(mesh);
    std::vector<double2> keps(m->nobj, make_double2(k_eps.re, k_eps.im));
    const bem::OsrcState &st = bem::osrc_get(m, pade_terms, theta, make_double2(k.re, k.im),
                                             keps, (hipStream_t)hip_stream);
    const bem::OsrcStats o = bem::osrc_stats(m, st);
    out->n_vertices = o.n;
    out->pade_terms = o.np;
    out->n_factors = o.nfactors;
    out->solves_per_apply = o.solves;
    out->nnz_l = o.nnz_l;
    out->nnz_offblock = o.nnz_ext;
    out->dense_entries = o.ndense;
    out->mass_nnz = o.mass_nnz;
    out->factor_bytes = o.factor_bytes;
    out->bytes_per_apply = o.bytes_per_apply;
    return BEM_OK;
    BEM_API_END
}

int pmchwt_rhs(const bem_mesh *mesh, bem_c64 k_ext, const double *directions, int n_waves,
               bem_c64 *f, void *hip_stream) {
    BEM_API_BEGIN
    check_mesh(mesh);
    check_k(k_ext, "k_ext");
    if (!directions || !f || n_waves < 1) fail(BEM_E_INVAL, "bad directions/f/n_waves");
    for (int w = 0; w < n_waves; w++) {
        const double *d = directions + 3 * w;
        double nrm = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (!(std::fabs(nrm - 1.0) < 1e-6)) fail(BEM_E_INVAL, "directions must be unit vectors");
    }
    bem::rhs_project(const_cast<bem_mesh *>(mesh), make_double2(k_ext.re, k_ext.im),
                     directions, n_waves, (double2 *)f, (hipStream_t)hip_stream);
    return BEM_OK;
    BEM_API_END
}

int bem_far_field(const bem_mesh *mesh, bem_c64 k_ext, const bem_c64 *solution,
                  const double *dirs, int n_dirs, bem_c64 *out, void *hip_stream) {
    BEM_API_BEGIN
    check_mesh(mesh);
    check_k(k_ext, "k_ext");
    if (!solution || !dirs || !out || n_dirs < 1) fail(BEM_E_INVAL, "bad arguments");
    bem::far_field_eval(const_cast<bem_mesh *>(mesh), make_double2(k_ext.re, k_ext.im),
                        (const double2 *)solution, dirs, n_dirs, (double2 *)out,
                        (hipStream_t)hip_stream);
    return BEM_OK;
    BEM_API_END
}

namespace {

int field_entry(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int, double rho,
                const bem::ObjMaterials *om, const double *direction, const bem_c64 *solution,
                const double *points, int64_t n_points, bem_c64 *out, int32_t *region,
                void *hip_stream) {
    BEM_API_BEGIN
    check_mesh(mesh);
    check_k(k_ext, "k_ext");
    check_k(k_int, "k_int");
    if (!(rho > 0) || !std::isfinite(rho)) fail(BEM_E_INVAL, "rho must be positive");
    if (n_points < 0) fail(BEM_E_INVAL, "n_points must be >= 0");
    if (!direction) fail(BEM_E_INVAL, "direction is NULL");
    const double *d = direction;
    if (!(std::fabs(std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) - 1.0) < 1e-6))
        fail(BEM_E_INVAL, "direction must be a unit vector");
    if (n_points == 0) return BEM_OK;
    if (!solution || !points || !out) fail(BEM_E_INVAL, "solution, points and out must be device pointers");
    if ((n_points + 255) / 256 > INT32_MAX) fail(BEM_E_INVAL, "n_points too large");
    bem::field_eval(const_cast<bem_mesh *>(mesh), make_double2(k_ext.re, k_ext.im),
                    make_double2(k_int.re, k_int.im), rho, d, (const double2 *)solution, points,
                    n_points, (double2 *)out, region, (hipStream_t)hip_stream, om);
    return BEM_OK;
    BEM_API_END
}

}   // namespace

int pmchwt_field(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int, double rho,
                 const double *direction, const bem_c64 *solution, const double *points,
                 int64_t n_points, bem_c64 *out, int32_t *region, void *hip_stream) {
    return field_entry(mesh, k_ext, k_int, rho, nullptr, direction, solution, points, n_points,
                       out, region, hip_stream);
}

int pmchwt_field_multi(const bem_mesh *mesh, bem_c64 k_ext, const bem_c64 *k_int,
                       const double *rho, const double *direction, const bem_c64 *solution,
                       const double *points, int64_t n_points, bem_c64 *out, int32_t *region,
                       void *hip_stream) {
    BEM_API_BEGIN
    const bem::ObjMaterials om = materials(mesh, k_int, rho);
    return field_entry(mesh, k_ext, k_int[0], rho[0], &om, direction, solution, points,
                       n_points, out, region, hip_stream);
    BEM_API_END
}

int bem_hmat_info(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int, double rho,
                  bem_hmat_stats *out, void *hip_stream) {
    BEM_API_BEGIN
    check_mesh(mesh);
    check_k(k_ext, "k_ext");
    check_k(k_int, "k_int");
    if (!(rho > 0) || !std::isfinite(rho)) fail(BEM_E_INVAL, "rho must be positive");
    if (!out) fail(BEM_E_INVAL, "out is NULL");
    bem_mesh *m = const_cast<bem_mesh *>(mesh);
    const bem::HMatStats &st =
        bem::hmat_stats(bem::hmat_get(m, make_double2(k_ext.re, k_ext.im),
                                      make_double2(k_int.re, k_int.im), rho,
                                      (hipStream_t)hip_stream));
    out->bytes = st.bytes;
    out->lowrank_bytes = st.lowrank_bytes;
    out->dense_bytes = st.dense_bytes;
    out->n_clusters = st.n_clusters;
    out->n_admissible = st.n_admissible;
    out->n_dense = st.n_dense;
    out->max_rank = st.max_rank;
    out->split_blocks = st.split_blocks;
    out->leaf = st.leaf;
    out->kmax = st.kmax;
    out->mean_rank = st.mean_rank;
    out->admissible_fraction = st.admissible_fraction;
    out->eta = st.eta;
    out->tol = st.tol;
    out->setup_seconds = st.setup_seconds;
    out->alpha = st.alpha;
    return BEM_OK;
    BEM_API_END
}

int bem_tune_set(const char *key, int64_t value) {
    BEM_API_BEGIN
    if (!key) fail(BEM_E_INVAL, "key is NULL");
    const std::string k(key);
    bem::Tuning &t = bem::tuning();
    if (k == "farfield.multi_max") {
        if (value != 1 && value != 2 && value != 4) fail(BEM_E_INVAL, "farfield.multi_max: 1, 2 or 4");
        t.farfield_multi_max = (int)value;
    } else if (k == "farfield.block") {
        if (value != 64 && value != 128 && value != 256) fail(BEM_E_INVAL, "farfield.block: 64, 128 or 256");
        t.farfield_block = (int)value;
    } else if (k == "farfield.sym_round_mib") {
        if (value < 1 || value > 65536) fail(BEM_E_INVAL, "farfield.sym_round_mib: 1..65536");
        t.farfield_sym_round_mib = (int)value;
    } else if (k == "farfield.symmetric") {
        if (value != 0 && value != 1) fail(BEM_E_INVAL, "farfield.symmetric: 0 or 1");
        t.farfield_symmetric = (int)value;
    } else if (k == "dense.skinny_min_rhs") {
        if (value < 2 || value > 1 << 20) fail(BEM_E_INVAL, "dense.skinny_min_rhs out of range");
        t.dense_skinny_min_rhs = (int)value;
    } else if (k == "dense.gemm_min_rhs") {
        if (value < 1 || value > 1 << 20) fail(BEM_E_INVAL, "dense.gemm_min_rhs out of range");
        t.dense_gemm_min_rhs = (int)value;
    } else if (k == "solve.refine_update") {
        if (value != 0 && value != 1) fail(BEM_E_INVAL, "solve.refine_update: 0 or 1");
        t.solve_refine_update = (int)value;
    } else if (k == "solve.residual_dense_gib") {
        if (value < 0 || value > 1024) fail(BEM_E_INVAL, "solve.residual_dense_gib: 0..1024");
        t.solve_residual_dense_gib = (int)value;
    } else if (k == "hmat.leaf") {
        if (value < 8 || value > 64) fail(BEM_E_INVAL, "hmat.leaf: 8..64");
        t.hmat_leaf = (int)value;
    } else if (k == "hmat.eta_pct") {
        if (value < 10 || value > 1000) fail(BEM_E_INVAL, "hmat.eta_pct: 10..1000");
        t.hmat_eta_pct = (int)value;
    } else if (k == "hmat.tol_ppb") {
        if (value < 100 || value > 100000000) fail(BEM_E_INVAL, "hmat.tol_ppb: 100..1e8");
        t.hmat_tol_ppb = value;
    } else if (k == "hmat.kmax") {
        if (value < 4 || value > 512) fail(BEM_E_INVAL, "hmat.kmax: 4..512");
        t.hmat_kmax = (int)value;
    } else if (k == "osrc.split") {
        if (value < 0 || value > 3) fail(BEM_E_INVAL, "osrc.split: 0, 1, 2 or 3");
        t.osrc_split = (int)value;
    } else if (k == "osrc.sub_rows") {
        if (value != 0 && (value < 64 || value > 8192)) fail(BEM_E_INVAL, "osrc.sub_rows: 0 or 64..8192");
        t.osrc_sub_rows = (int)value;
    } else if (k == "osrc.top_single_work") {
        if (value < 0 || value > (int64_t)1 << 30) fail(BEM_E_INVAL, "osrc.top_single_work out of range");
        t.osrc_top_single_work = (int)value;
    } else if (k == "osrc.bottom_rows") {
        if (value != 0 && (value < 64 || value > 8192)) fail(BEM_E_INVAL, "osrc.bottom_rows: 0 or 64..8192");
        t.osrc_bottom_rows = (int)value;
    } else {
        fail(BEM_E_INVAL, "unknown tuning key " + k);
    }
    return BEM_OK;
    BEM_API_END
}

int bem_tune_get(const char *key, int64_t *value) {
    BEM_API_BEGIN
    if (!key || !value) fail(BEM_E_INVAL, "key or value is NULL");
    const std::string k(key);
    bem::Tuning &t = bem::tuning();
    if (k == "farfield.multi_max") *value = t.farfield_multi_max;
    else if (k == "farfield.block") *value = t.farfield_block;
    else if (k == "farfield.symmetric") *value = t.farfield_symmetric;
    else if (k == "farfield.sym_round_mib") *value = t.farfield_sym_round_mib;
    else if (k == "dense.skinny_min_rhs") *value = t.dense_skinny_min_rhs;
    else if (k == "dense.gemm_min_rhs") *value = t.dense_gemm_min_rhs;
    else if (k == "solve.refine_update") *value = t.solve_refine_update;
    else if (k == "solve.residual_dense_gib") *value = t.solve_residual_dense_gib;
    else if (k == "hmat.leaf") *value = t.hmat_leaf;
    else if (k == "hmat.eta_pct") *value = t.hmat_eta_pct;
    else if (k == "hmat.tol_ppb") *value = t.hmat_tol_ppb;
    else if (k == "hmat.kmax") *value = t.hmat_kmax;
    else if (k == "osrc.split") *value = t.osrc_split;
    else if (k == "osrc.sub_rows") *value = t.osrc_sub_rows;
    else if (k == "osrc.top_single_work") *value = t.osrc_top_single_work;
    else if (k == "osrc.bottom_rows") *value = t.osrc_bottom_rows;
    else fail(BEM_E_INVAL, "unknown tuning key " + k);
    return BEM_OK;
    BEM_API_END
}

int bem_valu_rates(double *rates, void *hip_stream) {
    BEM_API_BEGIN
    if (!rates) fail(BEM_E_INVAL, "rates is NULL");
    bem::valu_rates(rates, (hipStream_t)hip_stream);
    return BEM_OK;
    BEM_API_END
}

int bem_profile_enable(int enable) {
    BEM_API_BEGIN
    std::lock_guard<std::mutex> g(bem::g_prof_mu);
    if (enable) bem::prof_clear_locked();
    bem::g_prof_on = enable != 0;
    return BEM_OK;
    BEM_API_END
}

int bem_profile_read(const char *kernel, double *total_ms, int64_t *launches) {
    BEM_API_BEGIN
    if (!kernel) fail(BEM_E_INVAL, "kernel name is NULL");
    std::lock_guard<std::mutex> g(bem::g_prof_mu);
    double ms = 0;
    int64_t n = 0;
    for (auto &r : bem::g_prof) {
        if (r.name != kernel) continue;
        BEM_HIP(hipEventSynchronize(r.b));
        float e = 0;
        BEM_HIP(hipEventElapsedTime(&e, r.a, r.b));
        ms += e;
        n++;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = n;
    return BEM_OK;
    BEM_API_END
}

}   // extern "C"

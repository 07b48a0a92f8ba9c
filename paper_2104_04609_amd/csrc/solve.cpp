// OSRC-preconditioned permuted PMCHWT solve (Sec. 2.7), strong form (mass
// preconditioning, Sec. 2.4), unrestarted GMRES from x_0 = 0 (Sec. 3.1):
//
//   P x = b,  P = L M^{-1} B,  b = L M^{-1} f,  L = diag(L_DtN, L_NtD) per object.
//
// The formulations it is compared with (Sec. 3.1) share the driver: standard
// PMCHWT and Mueller (Sec. 2.2) in strong form, and PMCHWT with the
// block-diagonal Calderon preconditioner (Sec. 2.5); see Op.
//
// The preconditioner is applied to the weak vector directly: L M^{-1} y uses
// M (M^{-1} y) = y, so no separate mass solve is needed.  GMRES runs in FP64:
// Arnoldi by classical Gram-Schmidt with one reorthogonalisation (CGS2) on the
// device, Givens rotations of the small Hessenberg matrix on the host.
//
// Precision form (BEM_FP32): iterative refinement.  The outer residual
// r = b - P64 x uses the FP64 pair kernel; the inner GMRES solves P32 d = r
// with the FP32 pair kernel (near field, OSRC and Arnoldi stay FP64) until its
// residual is below inner_tol * tol * ||b||, then x += d.
//
// Residual update: once a residual r_s = b - P64 x_s has been formed in FP64,
// the next one is r_{s+1} = r_s - P64 d = (r_s - P32 d) - (P64 - P32) d.  The
// correction d solves a system whose right-hand side is already small, so the
// FP32 operator's error on it, |(P64 - P32) d| <= eps |P32 d|, is far below
// the tolerance: r_s - P32 d is formed with one FP32 product and eps |P32 d|
// is carried as an error bound, added to the reported residual.  eps =
// REFINE_OP_BOUND is a hundred times the relative error measured for the FP32
// preconditioned operator on the workloads tested (about 1e-6).  When the
// carried bound would reach a tenth of the tolerance the residual is formed
// in FP64 again (tuning key "solve.refine_update" = 0 forms every residual in
// FP64).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>

#include "blas.h"
#include "osrc_internal.h"

namespace bem {

static thread_local ReserveHook t_reserve_hook = nullptr;
static thread_local void *t_reserve_ctx = nullptr;

ReserveScope::ReserveScope(ReserveHook hook, void *ctx)
    : prev_hook(t_reserve_hook), prev_ctx(t_reserve_ctx) {
    t_reserve_hook = hook;
    t_reserve_ctx = ctx;
}
ReserveScope::~ReserveScope() {
    t_reserve_hook = prev_hook;
    t_reserve_ctx = prev_ctx;
}
void reserve_bytes(int64_t delta) {
    if (t_reserve_hook) t_reserve_hook(t_reserve_ctx, delta);
}

namespace {

using cdd = std::complex<double>;

void copy_vec(double2 *dst, const double2 *src, int64_t n, hipStream_t s);

// Halves of each of R vectors [R][2N] exchanged: out_r = [in_r[N:]; in_r[:N]].
void swap_halves(const double2 *in, double2 *out, int64_t N, int R, hipStream_t s) {
    for (int r = 0; r < R; r++) {
        copy_vec(out + 2 * N * r, in + 2 * N * r + N, N, s);
        copy_vec(out + 2 * N * r + N, in + 2 * N * r, N, s);
    }
}

// P applied to R right-hand sides at once (contiguous [R][2N] in and out):
// weak operator (assembled or pair kernel + near field; the Mueller operator
// when the near field is Mueller's), then the preconditioner of the
// formulation.  OSRC: L M^{-1}.  The others are defined on the paper's
// ordering u = [phi; psi] (B~ u = B S u with S the half swap) while GMRES
// iterates on x = [psi; phi] = S u: they apply S P~ S, unitarily similar to
// P~, so the residual history is that of P~ on u.  PMCHWT and Mueller:
// P~ = M^{-1} B~, so S P~ S x = S M^{-1} B x.  Calderon: P~ = Q^2 with
// Q y = M^{-1} B S y (C = B~ for one object), so S P~ S x =
// S M^{-1} B S M^{-1} B x.
struct Op {
    bem_mesh *m;
    const NearOperator *nf;
    double2 k0, k1;
    double rho;
    OsrcState *st;
    hipStream_t s;
    int form = BEM_FORM_OSRC;
    const DenseOperator *dense = nullptr;   // assembled operator (FP32 form)
    const DenseOperator *dense64 = nullptr; // assembled complex128 operator (FP64 form, path 1)
    HMatrix *hm = nullptr;                  // compressed operator (FP32 form, path 3)
    const ObjMaterials *om = nullptr;       // per-object materials, or k1, rho for all
    DevBuf<double2> yw, t1, t2;              // weak-form scratch [R][2N]
    DevBuf<double2> px, py;                  // one object's entries [R][2 N_m]
    void weak(const double2 *in, double2 *out, int R, int precision) {
        if (precision == BEM_FP32_DENSE) {
            dense_apply(*dense, in, out, R, m->xs32, s);
        } else if (precision == BEM_FP32_HMAT) {
            for (int r = 0; r < R; r++) hmat_apply(*hm, m, *nf, in + r * 2 * m->N, out + r * 2 * m->N, s);
        } else if (precision == BEM_FP64 && dense64) {
            dense_apply(*dense64, in, out, R, m->xs32, s);
        } else {
            farfield_apply_batch(m, *nf, k0, k1, rho, in, out, R, precision, s);
        }
    }
    // C y of the block-diagonal Calderon preconditioner on x-ordered vectors:
    // the whole operator for one object; with several, each object's own
    // PMCHWT operator (its exterior self-interaction and interior operators)
    // on its own entries, through the object's mesh of its own
    void calderon_c(const double2 *in, double2 *out, int R, int precision) {
        if (m->nobj == 1) {
            weak(in, out, R, precision);
            return;
        }
        mesh_parts(m);
        for (int o = 0; o < m->nobj; o++) {
            bem_mesh *pm = m->parts[o].get();
            const int64_t nm = pm->N;
            if (px.n < (size_t)(2 * nm * R)) px.alloc((size_t)(2 * nm * R));
            if (py.n < (size_t)(2 * nm * R)) py.alloc((size_t)(2 * nm * R));
            gather_halves(in, m->part_vidx[o].p, m->N, nm, R, px.p, s);
            const double2 ko = om ? om->k[o] : k1;
            const double ro = om ? om->rho[o] : rho;
            if (precision == BEM_FP32_DENSE || (precision == BEM_FP64 && dense64)) {
                const bool f64 = precision == BEM_FP64;
                dense_apply(dense_get(pm, k0, ko, ro, s, 1, nullptr, f64), px.p, py.p, R,
                            pm->xs32, s);
            } else {
                const NearOperator &nfo = nearfield_get(pm, k0, ko, ro, s);
                farfield_apply_batch(pm, nfo, k0, ko, ro, px.p, py.p, R, precision, s);
            }
            scatter_halves(py.p, m->part_vidx[o].p, m->N, nm, R, out, s);
        }
    }
    // the preconditioner on a weak-form vector yw -> out; `precision` is the
    // operator precision of the second application (Calderon)
    void precondition(const double2 *w, double2 *out, int R, int precision) {
        const int64_t n2 = 2 * m->N;
        if (form == BEM_FORM_OSRC) {
            osrc_apply_from_weak(m, *st, w, out, R, s);
        } else if (form == BEM_FORM_PMCHWT || form == BEM_FORM_MULLER) {
            if (t1.n < (size_t)(R * n2)) t1.alloc((size_t)(R * n2));
            osrc_mass_solve(m, *st, w, t1.p, 2 * R, s);
            swap_halves(t1.p, out, m->N, R, s);
        } else {
            if (t1.n < (size_t)(R * n2)) t1.alloc((size_t)(R * n2));
            if (t2.n < (size_t)(R * n2)) t2.alloc((size_t)(R * n2));
            osrc_mass_solve(m, *st, w, t1.p, 2 * R, s);
            swap_halves(t1.p, t2.p, m->N, R, s);
            calderon_c(t2.p, t1.p, R, precision);
            osrc_mass_solve(m, *st, t1.p, t2.p, 2 * R, s);
            swap_halves(t2.p, out, m->N, R, s);
        }
    }
    void apply(const double2 *in, double2 *out, int R, int precision) {
        const int64_t n2 = 2 * m->N;
        if (yw.n < (size_t)(R * n2)) yw.alloc((size_t)(R * n2));
        weak(in, yw.p, R, precision);
        precondition(yw.p, out, R, precision);
    }
};

// Initial Krylov basis capacity (vectors beyond v_0); the basis doubles as it
// fills.
constexpr int KRYLOV_CAP0 = 64;

struct Workspace {
    int64_t n2 = 0;
    int cap = 0;               // basis vectors beyond v_0
    DevBuf<double2> V;         // [cap + 1][n2]
    DevBuf<double2> h;         // [2 (cap + 1) + 1]
    void ensure(int need, hipStream_t s) {   // need = number of vectors
        if (need <= cap + 1) return;
        int ncap = std::max(need - 1, std::max(2 * cap, KRYLOV_CAP0));
        // growth beyond the initial capacity is reported (the new basis is
        // held beside the old one while it is copied)
        const int64_t vb = n2 * (int64_t)sizeof(double2);
        if (V.p) reserve_bytes((int64_t)(ncap + 1) * vb);
        DevBuf<double2> nv((size_t)(ncap + 1) * n2);
        if (V.p) BEM_HIP(hipMemcpyAsync(nv.p, V.p, (size_t)(cap + 1) * n2 * sizeof(double2),
                                        hipMemcpyDeviceToDevice, s));
        BEM_HIP(hipStreamSynchronize(s));
        const int64_t old = V.p ? (int64_t)(cap + 1) * vb : 0;
        V = std::move(nv);
        if (old) reserve_bytes(-old);
        h.alloc(2 * (size_t)(ncap + 1) + 1);
        cap = ncap;
    }
};



// Squared norms of R vectors (stride n) into host nrm[R] (one sync).
void dev_norms(const double2 *v, int64_t n, int R, double2 *dbuf, double *nrm, hipStream_t s) {
    DevBuf<double2> part((size_t)std::min(R, BLAS_MAX_BATCH) * blas_dot_chunks(n));
    for (int r0 = 0; r0 < R; r0 += BLAS_MAX_BATCH) {
        const int A = std::min(BLAS_MAX_BATCH, R - r0);
        CVecs x{};
        Vecs h{};
        for (int a = 0; a < A; a++) {
            x.p[a] = v + (r0 + a) * n;
            h.p[a] = dbuf + r0 + a;
        }
        blas_block_dot_batch(x, n, 1, x, n, h, A, part.p, s);
    }
    std::vector<double2> h(R);
    BEM_HIP(hipMemcpyAsync(h.data(), dbuf, R * sizeof(double2), hipMemcpyDeviceToHost, s));
    BEM_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < R; r++) {
        if (!std::isfinite(h[r].x)) fail(BEM_E_NAN, "NaN/Inf in a vector norm");
        nrm[r] = std::sqrt(std::max(h[r].x, 0.0));
    }
}

void copy_vec(double2 *dst, const double2 *src, int64_t n, hipStream_t s) {
    BEM_HIP(hipMemcpyAsync(dst, src, n * sizeof(double2), hipMemcpyDeviceToDevice, s));
}

// Waves solved together in one lockstep group.
constexpr int SOLVE_BATCH = 16;
static_assert(SOLVE_BATCH <= BLAS_MAX_BATCH, "lockstep groups are orthogonalised per launch");

// Bound on |(P64 - P32) v| / |P32 v| for the FP32 preconditioned operator
// used when a refinement residual is updated with the FP32 product.
constexpr double REFINE_OP_BOUND = 1e-4;

// Unrestarted GMRES for R systems op(x_r) = b_r from x_0 = 0, run in
// lockstep: every iteration applies the operator to the newest Krylov vector
// of all systems still running, then orthogonalises each system's vector
// against its own basis (CGS2 on the device, Givens on the host).  System r
// stops when |g_{j+1}| <= tol[r] ||b_r|| or after maxit[r] iterations.
// b, x: [R][n2].  Writes x, iters[r]; conv[r] = converged.
void gmres_batch(Op &op, int prec, const double2 *b, double2 *x, int R, int64_t n2,
                 const double *tol, const int *maxit, std::vector<Workspace> &ws,
                 int *iters, bool *conv, int *napply, hipStream_t s) {
    struct Sys {
        std::vector<cdd> H, cs, sn, g;
        double beta = 0;
        int m = 0;
        bool run = false;
    };
    std::vector<Sys> sy(R);
    if ((int)ws.size() < R) ws.resize(R);
    DevBuf<double2> nb(R);
    std::vector<double> bn(R);
    for (int r = 0; r < R; r++) {
        ws[r].n2 = n2;
        ws[r].ensure(2, s);
        BEM_HIP(hipMemsetAsync(x + r * n2, 0, n2 * sizeof(double2), s));
    }
    dev_norms(b, n2, R, nb.p, bn.data(), s);
    for (int r = 0; r < R; r++) {
        iters[r] = 0;
        conv[r] = bn[r] == 0.0;
        sy[r].beta = bn[r];
        sy[r].g.assign(1, cdd(bn[r]));
        sy[r].run = !conv[r] && maxit[r] > 0;
        if (sy[r].run)
            blas_axpby(make_double2(1.0 / bn[r], 0.0), b + r * n2, make_double2(0, 0), nullptr,
                       ws[r].V.p, n2, s);
    }
    DevBuf<double2> vin, vout, part;
    std::vector<double2> hh;
    const int64_t nch = blas_dot_chunks(n2);
    for (int j = 0;; j++) {
        std::vector<int> act;
        for (int r = 0; r < R; r++)
            if (sy[r].run) act.push_back(r);
        if (act.empty()) break;
        const int A = (int)act.size();   // <= SOLVE_BATCH = BLAS_MAX_BATCH
        if (vin.n < (size_t)(A * n2)) {
            vin.alloc((size_t)(A * n2));
            vout.alloc((size_t)(A * n2));
        }
        if (part.n < (size_t)(A * (j + 1) * nch))   // grows with the basis, doubling
            part.alloc((size_t)(A * nch) * std::max(2 * (j + 1), 64));
        for (int a = 0; a < A; a++) ws[act[a]].ensure(j + 2, s);
        // every active system's newest vector through the operator, then CGS2
        // of each against its own basis, all systems per launch
        CVecs V{}, Vn_c{}, h1_c{}, h2_c{}, nr_c{}, vo{};
        Vecs Vn{}, h1{}, h2{}, nr{}, vi{};
        for (int a = 0; a < A; a++) {
            Workspace &w = ws[act[a]];
            V.p[a] = w.V.p;
            Vn.p[a] = w.V.p + (size_t)(j + 1) * n2;
            Vn_c.p[a] = Vn.p[a];
            vi.p[a] = vin.p + a * n2;
            vo.p[a] = vout.p + a * n2;
            h1.p[a] = w.h.p;
            h2.p[a] = w.h.p + (j + 1);
            nr.p[a] = w.h.p + 2 * (j + 1);
            h1_c.p[a] = h1.p[a];
            h2_c.p[a] = h2.p[a];
            nr_c.p[a] = nr.p[a];
        }
        CVecs vj{};
        for (int a = 0; a < A; a++) vj.p[a] = V.p[a] + (size_t)j * n2;
        blas_copy_batch(vi, vj, n2, A, s);
        op.apply(vin.p, vout.p, A, prec);
        blas_copy_batch(Vn, vo, n2, A, s);
        blas_block_dot_batch(V, n2, j + 1, Vn_c, n2, h1, A, part.p, s);
        blas_block_axpy_batch(V, n2, h1_c, j + 1, -1.0, Vn, n2, A, s);
        blas_block_dot_batch(V, n2, j + 1, Vn_c, n2, h2, A, part.p, s);
        blas_block_axpy_batch(V, n2, h2_c, j + 1, -1.0, Vn, n2, A, s);
        blas_block_dot_batch(Vn_c, n2, 1, Vn_c, n2, nr, A, part.p, s);
        blas_normalize_batch(Vn, nr_c, n2, A, s);
        for (int a = 0; a < A; a++) napply[act[a]]++;
        const size_t per = 2 * (size_t)(j + 1) + 1;
        hh.resize(per * A);
        for (int a = 0; a < A; a++)
            BEM_HIP(hipMemcpyAsync(hh.data() + a * per, ws[act[a]].h.p, per * sizeof(double2),
                                   hipMemcpyDeviceToHost, s));
        BEM_HIP(hipStreamSynchronize(s));
        for (int a = 0; a < A; a++) {
            const int r = act[a];
            Sys &q = sy[r];
            const double2 *h = hh.data() + a * per;
            // column j of the Hessenberg matrix (length j + 2)
            std::vector<cdd> col(j + 2);
            for (int i = 0; i <= j; i++)
                col[i] = cdd(h[i].x + h[j + 1 + i].x, h[i].y + h[j + 1 + i].y);
            const double hn = std::sqrt(std::max(h[2 * (j + 1)].x, 0.0));
            if (!std::isfinite(hn)) fail(BEM_E_NAN, "NaN/Inf in the Arnoldi process");
            col[j + 1] = hn;
            for (int i = 0; i < j; i++) {   // previous rotations
                cdd u = col[i], v = col[i + 1];
                col[i] = std::conj(q.cs[i]) * u + std::conj(q.sn[i]) * v;
                col[i + 1] = -q.sn[i] * u + q.cs[i] * v;
            }
            const double d = std::sqrt(std::norm(col[j]) + std::norm(col[j + 1]));
            cdd c0 = d > 0 ? col[j] / d : cdd(1.0), s0 = d > 0 ? col[j + 1] / d : cdd(0.0);
            q.cs.push_back(c0);
            q.sn.push_back(s0);
            col[j] = std::conj(c0) * col[j] + std::conj(s0) * col[j + 1];
            q.g.push_back(-s0 * q.g[j]);
            q.g[j] = std::conj(c0) * q.g[j];
            q.H.insert(q.H.end(), col.begin(), col.begin() + (j + 1));   // R column j
            q.m = j + 1;
            const double est = std::abs(q.g[j + 1]) / q.beta;
            if (!std::isfinite(est)) fail(BEM_E_NAN, "NaN/Inf in the GMRES residual");
            if (est <= tol[r]) {
                conv[r] = true;
                q.run = false;
            } else if (q.m >= maxit[r]) {
                q.run = false;
            }
        }
    }
    // x_r = V_r y_r with R_r y_r = g_r (back substitution, packed columns)
    for (int r = 0; r < R; r++) {
        Sys &q = sy[r];
        iters[r] = q.m;
        if (q.m == 0) continue;
        const int m = q.m;
        std::vector<cdd> y(m);
        auto Rm = [&](int i, int jj) { return q.H[(size_t)jj * (jj + 1) / 2 + i]; };
        for (int i = m - 1; i >= 0; i--) {
            cdd acc = q.g[i];
            for (int jj = i + 1; jj < m; jj++) acc -= Rm(i, jj) * y[jj];
            y[i] = acc / Rm(i, i);
        }
        std::vector<double2> yd(m);
        for (int i = 0; i < m; i++) yd[i] = make_double2(y[i].real(), y[i].imag());
        BEM_HIP(hipMemcpyAsync(ws[r].h.p, yd.data(), m * sizeof(double2), hipMemcpyHostToDevice,
                               s));
        blas_block_axpy(ws[r].V.p, n2, ws[r].h.p, m, 1.0, x + r * n2, n2, s);
        BEM_HIP(hipStreamSynchronize(s));
    }
}

double2 damped(double2 k, double R) {
    // k_eps = k (1 + 0.4 i (k R)^{-2/3}), principal branch (Sec. 2.6)
    cdd kk(k.x, k.y);
    cdd ke = kk * (1.0 + cdd(0, 0.4) * std::pow(kk * R, -2.0 / 3.0));
    return make_double2(ke.real(), ke.imag());
}

}   // namespace

void solve_check(const bem_mesh *m, double2 k0, double2 k1, double rho, const double *dirs,
                 int n_waves, double tol, const bem_solve_opts &o) {
    if (!m) fail(BEM_E_INVAL, "mesh is NULL");
    if (!dirs || n_waves < 1) fail(BEM_E_INVAL, "bad directions");
    if (!(tol > 0) || !std::isfinite(tol)) fail(BEM_E_INVAL, "tol must be positive");
    if (!(rho > 0) || !std::isfinite(rho)) fail(BEM_E_INVAL, "rho must be positive");
    for (double2 k : {k0, k1})
        if (!std::isfinite(k.x) || !std::isfinite(k.y) || k.y < 0 || (k.x == 0 && k.y == 0))
            fail(BEM_E_INVAL, "wavenumbers must be finite, nonzero, Im k >= 0");
    if (o.pade_terms < 1 || o.pade_terms > PADE_MAX) fail(BEM_E_INVAL, "pade_terms");
    if (o.precision != BEM_FP64 && o.precision != BEM_FP32) fail(BEM_E_INVAL, "precision");
    if (o.maxiter < 1 || o.max_outer < 1 || !(o.inner_tol > 0)) fail(BEM_E_INVAL, "opts");
    if (o.path < 0 || o.path > 3) fail(BEM_E_INVAL, "path must be 0, 1, 2 or 3");
    if (o.path == 3 && o.precision != BEM_FP32)
        fail(BEM_E_INVAL, "path 3 (compressed operator) serves the FP32 form's inner solves");
    if (o.path == 3 && o.formulation == BEM_FORM_CALDERON && m->nobj > 1)
        fail(BEM_E_UNSUPPORTED, "path 3: the Calderon preconditioner of several objects");
    if (o.formulation < BEM_FORM_OSRC || o.formulation > BEM_FORM_MULLER)
        fail(BEM_E_INVAL, "formulation must be 0, 1, 2 or 3");
    for (int w = 0; w < n_waves; w++) {
        const double *d = dirs + 3 * w;
        if (!(std::fabs(std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) - 1.0) < 1e-6))
            fail(BEM_E_INVAL, "directions must be unit vectors");
    }
}

void check_materials(const bem_mesh *m, const ObjMaterials &om) {
    if ((int)om.k.size() != m->nobj || (int)om.rho.size() != m->nobj)
        fail(BEM_E_INVAL, "one interior wavenumber and density ratio per object expected");
    for (int o = 0; o < m->nobj; o++) {
        const double2 k = om.k[o];
        if (!std::isfinite(k.x) || !std::isfinite(k.y) || k.y < 0 || (k.x == 0 && k.y == 0))
            fail(BEM_E_INVAL, "wavenumbers must be finite, nonzero, Im k >= 0");
        if (!(om.rho[o] > 0) || !std::isfinite(om.rho[o])) fail(BEM_E_INVAL, "rho must be positive");
    }
}

// The assembled FP32 path takes its FP64 residuals with the complex128
// operator (assembled once, the complex64 one rounded from it) when that
// operator is at most "solve.residual_dense_gib" GiB; a rule on the mesh and
// options alone, so that a result never depends on memory in use.
static bool residual_dense(const bem_mesh *m, const bem_solve_opts &o) {
    const int64_t lim = (int64_t)tuning().solve_residual_dense_gib.load() << 30;
    return o.precision == BEM_FP32 && lim > 0 && dense_bytes(m, true) <= lim &&
           (o.formulation != BEM_FORM_CALDERON || m->nobj == 1);
}

// Device bytes the assembled path of these options allocates: the operators
// it assembles (complex128 and its complex64 rounding, complex128, or
// complex64) with the assembly scratch and, for the Calderon preconditioner
// of several objects, each object's own operator and scratch.
static int64_t dense_path_need(const bem_mesh *m, const bem_solve_opts &o) {
    const bool f64 = o.precision == BEM_FP64, rd = residual_dense(m, o);
    int64_t b = f64 || rd ? dense_bytes(m, true) +
                                std::max(dense_assembly_scratch_bytes(m, true),
                                         rd ? dense_bytes(m) : (int64_t)0)
                          : dense_bytes(m) + dense_assembly_scratch_bytes(m);
    if (o.formulation == BEM_FORM_CALDERON && m->nobj > 1)
        for (int ob = 0; ob < m->nobj; ob++) {
            const int64_t No = std::count(m->vobj.begin(), m->vobj.end(), ob);
            const int64_t To = std::count(m->tobj.begin(), m->tobj.end(), ob);
            b += dense_need_bytes(No, To, f64);
        }
    return b;
}

int64_t solve_footprint(bem_mesh *m, double2 k0, double2 k1, double rho,
                        const bem_solve_opts &o, int n_waves) {
    (void)rho;
    const int64_t n2 = 2 * m->N, c16 = (int64_t)sizeof(double2);
    const int G = std::min(n_waves, SOLVE_BATCH);
    int64_t b = 4 * m->nf_nnz * c16;                          // near-field CSR values
    b += osrc_state_bytes(m, o.pade_terms, G);                 // OSRC factors + batch buffers
    const bool dense = o.precision == BEM_FP32 && o.path == 1;
    const bool rdense = dense && residual_dense(m, o);
    // the pair kernel's scratch unless every product is assembled
    const bool matrix_free = !(o.path == 1 && (o.precision == BEM_FP64 || rdense));
    if (matrix_free) {
        b += farfield_scratch_bytes(m, BEM_FP64, k0, k1, G);
        if (o.precision == BEM_FP32 && !dense)
            b += farfield_scratch_bytes(m, BEM_FP32, k0, k1, G);   // dyn32 beside dyn64
    }
    if (o.path == 1) b += dense_path_need(m, o);
    if (o.path == 3) b += hmat_bytes_estimate(m, k0, k1, rho);
    if (dense) b += 2 * G * n2 * 8 + dense_gemm_scratch_bytes(m, G);
    b += ((int64_t)n_waves + 8 * (int64_t)G) * n2 * c16;      // f, B, X, R, D, T, yw, vin, vout
    if (o.formulation == BEM_FORM_CALDERON) {
        b += 2 * (int64_t)G * n2 * c16;                       // t1, t2
        if (m->nobj > 1) b += 4 * m->nf_nnz * c16 + G * n2 * c16;   // parts: near fields, px, py
    }
    else if (o.formulation != BEM_FORM_OSRC) b += (int64_t)G * n2 * c16;       // t1
    // the initial Krylov basis; its growth is reported through reserve_bytes
    b += G * ((int64_t)(KRYLOV_CAP0 + 1) * n2 * c16 + (2 * (int64_t)o.maxiter + 8) * c16);
    // partial dot products of the orthogonalisation
    b += G * blas_dot_chunks(n2) * (2 * (int64_t)o.maxiter + 64) * c16;
    return b;
}

int solve_run(bem_mesh *m, double2 k0, double2 k1, double rho, const double *directions,
              int n_waves, double tol, const bem_solve_opts &o, double2 *solution,
              bem_solve_info *info, hipStream_t s, const ObjMaterials *om) {
    solve_check(m, k0, k1, rho, directions, n_waves, tol, o);
    if (om) check_materials(m, *om);
    if (!solution) fail(BEM_E_INVAL, "solution is NULL");
    const int64_t n2 = 2 * m->N;
    const int s1 = o.formulation == BEM_FORM_MULLER ? -1 : 1;   // Mueller operator
    const NearOperator &nf = nearfield_get(m, k0, k1, rho, s, s1, om);
    // OSRC wavenumber of each object: its interior one, or the exterior one
    std::vector<double2> ko(m->nobj, o.osrc_interior ? k1 : k0);
    if (om && o.osrc_interior) ko = om->k;
    std::vector<double2> keps(m->nobj);
    for (int ob = 0; ob < m->nobj; ob++)
        keps[ob] = damped(ko[ob], o.R > 0 ? o.R : 0.1 * m->obj_radius[ob]);
    OsrcState &st = osrc_get(m, o.pade_terms, o.theta, ko[0], keps, s, &ko);

    DevBuf<double2> f((size_t)n_waves * n2);
    rhs_project(m, k0, directions, n_waves, f.p, s);
    Op op{m, &nf, k0, k1, rho, &st, s};
    op.form = o.formulation;
    op.om = om;
    int inner = BEM_FP32;
    std::shared_ptr<const DenseOperator> dense_hold, dense_hold64;   // shared operators held
    if (o.path == 3) {
        op.hm = &hmat_get(m, k0, k1, rho, s, s1, om);
        inner = BEM_FP32_HMAT;
    } else if (o.path != 0) {
        const bool f64 = o.precision == BEM_FP64;
        bool use = o.path == 1;
        if (o.path == 2) {   // autotuned choice, else dense when it fits with room to spare
            size_t free_b = 0, total_b = 0;
            BEM_HIP(hipMemGetInfo(&free_b, &total_b));
            const bool rd = residual_dense(m, o);
            const int64_t need = dense_path_need(m, o) + (int64_t)(1ll << 30);
            const bool fits = need < (int64_t)free_b ||
                              !(f64  ? m->dense64_cache.empty()
                                : rd ? m->dense_rounded_cache.empty()
                                     : m->dense_cache.empty());
            // the autotuned table times the FP32 products (pair kernel against
            // complex64 operator): it decides FP32 solves only
            TuneEntry te;
            use = fits && !(o.precision == BEM_FP32 &&
                            tune_find(m->T, std::min(n_waves, SOLVE_BATCH), &te) && te.path == 0);
        }
        try {
            if (use && f64) {
                if (m->dense_share) {
                    dense_hold = dense_share_get(m, k0, k1, rho, s, s1, om, DENSE_C128);
                    op.dense64 = dense_hold.get();
                } else {
                    op.dense64 = &dense_get(m, k0, k1, rho, s, s1, om, true);
                }
            } else if (use && residual_dense(m, o)) {
                // FP32 form whose FP64 residuals use the complex128 operator: the
                // complex64 one is its rounding (one FP64 assembly)
                if (m->dense_share) {
                    dense_hold64 = dense_share_get(m, k0, k1, rho, s, s1, om, DENSE_C128);
                    dense_hold = dense_share_get(m, k0, k1, rho, s, s1, om, DENSE_C64_ROUNDED);
                    op.dense64 = dense_hold64.get();
                    op.dense = dense_hold.get();
                } else {
                    op.dense64 = &dense_get(m, k0, k1, rho, s, s1, om, true);
                    op.dense = &dense_get_rounded(m, k0, k1, rho, s, s1, om);
                }
                inner = BEM_FP32_DENSE;
            } else if (use) {
                if (m->dense_share) {
                    dense_hold = dense_share_get(m, k0, k1, rho, s, s1, om, DENSE_C64);
                    op.dense = dense_hold.get();
                } else {
                    op.dense = &dense_get(m, k0, k1, rho, s, s1, om);
                }
                inner = BEM_FP32_DENSE;
            }
        } catch (const Error &e) {
            // the automatic path falls back to the matrix-free operator when
            // the assembled one does not fit after all
            if (o.path != 2 || e.code != BEM_E_NOMEM) throw;
            (void)hipGetLastError();
            dense_hold.reset();
            dense_hold64.reset();
            op.dense = op.dense64 = nullptr;
            inner = BEM_FP32;
        }
    }
    // waves are solved in lockstep groups of up to SOLVE_BATCH
    const int G = std::min(n_waves, SOLVE_BATCH);
    DevBuf<double2> B((size_t)G * n2), X((size_t)G * n2), Rv((size_t)G * n2),
        D((size_t)G * n2), T((size_t)G * n2), nb(G);
    std::vector<Workspace> ws;
    int worst = BEM_OK;
    for (int w0 = 0; w0 < n_waves; w0 += G) {
        const int R = std::min(G, n_waves - w0);
        const auto t0 = std::chrono::steady_clock::now();
        std::vector<int> n64(R, 0), n32(R, 0), its(R, 0), outer(R, 0);
        std::vector<double> bn(R), rel(R, 0.0);
        std::vector<char> cv(R, 0);
        op.precondition(f.p + (size_t)w0 * n2, B.p, R, BEM_FP64);
        dev_norms(B.p, n2, R, nb.p, bn.data(), s);
        if (o.precision == BEM_FP64) {
            std::vector<double> tl(R, tol);
            std::vector<int> mi(R, o.maxiter);
            bool cvb[SOLVE_BATCH];
            gmres_batch(op, BEM_FP64, B.p, X.p, R, n2, tl.data(), mi.data(), ws, its.data(), cvb,
                        n64.data(), s);
            // true residual with the FP64 operator
            op.apply(X.p, Rv.p, R, BEM_FP64);
            blas_axpby(make_double2(1, 0), B.p, make_double2(-1, 0), Rv.p, Rv.p, R * n2, s);
            std::vector<double> rn(R);
            dev_norms(Rv.p, n2, R, nb.p, rn.data(), s);
            for (int r = 0; r < R; r++) {
                n64[r]++;
                outer[r] = 1;
                rel[r] = bn[r] > 0 ? rn[r] / bn[r] : 0.0;
                cv[r] = cvb[r] || rel[r] <= tol;
            }
        } else {
            // iterative refinement: x += d, P32 d = r to eta ||b||, r = b - P64 x
            // (or r -= P32 d with its error bound carried, see the header)
            BEM_HIP(hipMemsetAsync(X.p, 0, R * n2 * sizeof(double2), s));
            copy_vec(Rv.p, B.p, R * n2, s);
            std::vector<double> rn(bn), carried(R, 0.0);
            std::vector<char> exact(R, 0);   // Rv holds an FP64 residual of X (+ updates)
            const bool update = tuning().solve_refine_update.load() != 0;
            for (int r = 0; r < R; r++) rel[r] = bn[r] > 0 ? 1.0 : 0.0;
            for (;;) {
                std::vector<int> act;
                for (int r = 0; r < R; r++)
                    if (rel[r] > tol && outer[r] < o.max_outer && its[r] < o.maxiter)
                        act.push_back(r);
                if (act.empty()) break;
                const int A = (int)act.size();
                std::vector<double> eta(A);
                std::vector<int> mi(A), it(A), na(A, 0);
                bool cvb[SOLVE_BATCH];
                for (int a = 0; a < A; a++) {
                    const int r = act[a];
                    eta[a] = std::min(0.5, o.inner_tol * tol * bn[r] / rn[r]);
                    mi[a] = o.maxiter - its[r];
                    copy_vec(T.p + a * n2, Rv.p + act[a] * n2, n2, s);
                }
                gmres_batch(op, inner, T.p, D.p, A, n2, eta.data(), mi.data(), ws, it.data(),
                            cvb, na.data(), s);
                for (int a = 0; a < A; a++) {
                    const int r = act[a];
                    its[r] += it[a];
                    outer[r]++;
                    n32[r] += na[a];
                    blas_axpby(make_double2(1, 0), X.p + r * n2, make_double2(1, 0),
                               D.p + a * n2, X.p + r * n2, n2, s);
                }
                // systems whose residual is updated with the FP32 product of d,
                // the others formed in FP64 from x
                std::vector<int> upd, full;
                for (int a = 0; a < A; a++) {
                    const int r = act[a];
                    // (the bound on P32's error holds for the pair kernel and the
                    // assembled operators, not for the compressed one)
                    const bool cheap = update && inner != BEM_FP32_HMAT && exact[r] &&
                                       carried[r] + REFINE_OP_BOUND * rn[r] <= 0.1 * tol * bn[r];
                    (cheap ? upd : full).push_back(a);
                }
                if (!upd.empty()) {
                    // D holds d of every active system (slot a): first, before
                    // the FP64 products below overwrite it; T gets P32 d
                    const int U = (int)upd.size();
                    for (int u = 0; u < U; u++) copy_vec(T.p + u * n2, D.p + upd[u] * n2, n2, s);
                    op.apply(T.p, D.p, U, inner);
                    std::vector<double> pn(U), nrm(U);
                    dev_norms(D.p, n2, U, nb.p, pn.data(), s);
                    for (int u = 0; u < U; u++) {
                        const int r = act[upd[u]];
                        n32[r]++;
                        blas_axpby(make_double2(1, 0), Rv.p + r * n2, make_double2(-1, 0),
                                   D.p + u * n2, Rv.p + r * n2, n2, s);
                        copy_vec(T.p + u * n2, Rv.p + r * n2, n2, s);
                    }
                    dev_norms(T.p, n2, U, nb.p, nrm.data(), s);
                    for (int u = 0; u < U; u++) {
                        const int r = act[upd[u]];
                        carried[r] += REFINE_OP_BOUND * pn[u];
                        rn[r] = nrm[u];
                        rel[r] = (rn[r] + carried[r]) / bn[r];
                    }
                }
                if (!full.empty()) {
                    const int F = (int)full.size();
                    for (int f = 0; f < F; f++)
                        copy_vec(T.p + f * n2, X.p + act[full[f]] * n2, n2, s);
                    op.apply(T.p, D.p, F, BEM_FP64);
                    for (int f = 0; f < F; f++) {
                        const int r = act[full[f]];
                        n64[r]++;
                        blas_axpby(make_double2(1, 0), B.p + r * n2, make_double2(-1, 0),
                                   D.p + f * n2, Rv.p + r * n2, n2, s);
                        copy_vec(T.p + f * n2, Rv.p + r * n2, n2, s);
                    }
                    std::vector<double> nrm(F);
                    dev_norms(T.p, n2, F, nb.p, nrm.data(), s);
                    for (int f = 0; f < F; f++) {
                        const int r = act[full[f]];
                        exact[r] = 1;
                        carried[r] = 0.0;
                        rn[r] = nrm[f];
                        rel[r] = rn[r] / bn[r];
                    }
                }
            }
            for (int r = 0; r < R; r++) cv[r] = rel[r] <= tol;
        }
        copy_vec(solution + (size_t)w0 * n2, X.p, R * n2, s);
        BEM_HIP(hipStreamSynchronize(s));
        const double secs =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int r = 0; r < R; r++) {
            if (info) {
                bem_solve_info &q = info[w0 + r];
                q.iterations = its[r];
                q.outer_steps = outer[r];
                q.fp64_matvecs = n64[r];
                q.fp32_matvecs = n32[r];
                q.rel_residual = rel[r];
                q.seconds = secs;
            }
            if (!cv[r]) worst = BEM_W_NOT_CONVERGED;
        }
    }
    return worst;
}

}   // namespace bem

using bem::fail;

extern "C" {

void bem_solve_opts_default(bem_solve_opts *o) {
    if (!o) return;
    o->pade_terms = 4;
    o->theta = M_PI / 3;
    o->osrc_interior = 1;
    o->R = 0;
    o->precision = BEM_FP64;
    o->maxiter = 1000;
    o->inner_tol = 0.6;
    o->max_outer = 8;
    o->path = 2;
    o->formulation = BEM_FORM_OSRC;
}

namespace {

int solve_entry(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int, double rho,
                const bem::ObjMaterials *om, const double *directions, int n_waves, double tol,
                const bem_solve_opts *opts_in, bem_c64 *solution, bem_solve_info *info,
                void *hip_stream) {
    try {
        if (!mesh) fail(BEM_E_INVAL, "mesh is NULL");
        if (!directions || !solution || n_waves < 1) fail(BEM_E_INVAL, "bad directions/solution");
        bem_solve_opts o;
        bem_solve_opts_default(&o);
        if (opts_in) o = *opts_in;
        return bem::solve_run(const_cast<bem_mesh *>(mesh), make_double2(k_ext.re, k_ext.im),
                              make_double2(k_int.re, k_int.im), rho, directions, n_waves, tol, o,
                              (double2 *)solution, info, (hipStream_t)hip_stream, om);
    } catch (const bem::Error &e) {
        bem::set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        bem::set_last_error("host allocation failed");
        return BEM_E_NOMEM;
    }
}

}   // namespace

int pmchwt_solve(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int, double rho,
                 const double *directions, int n_waves, double tol,
                 const bem_solve_opts *opts_in, bem_c64 *solution, bem_solve_info *info,
                 void *hip_stream) {
    return solve_entry(mesh, k_ext, k_int, rho, nullptr, directions, n_waves, tol, opts_in,
                       solution, info, hip_stream);
}

int pmchwt_solve_multi(const bem_mesh *mesh, bem_c64 k_ext, const bem_c64 *k_int,
                       const double *rho, const double *directions, int n_waves, double tol,
                       const bem_solve_opts *opts_in, bem_c64 *solution, bem_solve_info *info,
                       void *hip_stream) {
    if (!mesh || !k_int || !rho) {
        bem::set_last_error("mesh, k_int and rho must not be NULL");
        return BEM_E_INVAL;
    }
    bem::ObjMaterials om;
    for (int ob = 0; ob < mesh->nobj; ob++) {
        om.k.push_back(make_double2(k_int[ob].re, k_int[ob].im));
        om.rho.push_back(rho[ob]);
    }
    return solve_entry(mesh, k_ext, k_int[0], rho[0], &om, directions, n_waves, tol, opts_in,
                       solution, info, hip_stream);
}

}   // extern "C"

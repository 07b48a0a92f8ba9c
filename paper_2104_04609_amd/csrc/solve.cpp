// OSRC-preconditioned permuted PMCHWT solve (Sec. 2.7), strong form (mass
// preconditioning, Sec. 2.4), unrestarted GMRES from x_0 = 0 (Sec. 3.1):
//
//   P x = b,  P = L M^{-1} B,  b = L M^{-1} f,  L = diag(L_DtN, L_NtD) per object.
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
#include <chrono>
#include <cmath>
#include <complex>

#include "blas.h"
#include "osrc_internal.h"

namespace bem {

namespace {

using cdd = std::complex<double>;

struct Op {
    bem_mesh *m;
    const NearOperator *nf;
    double2 k0, k1;
    double rho;
    OsrcState *st;
    hipStream_t s;
    double2 *yw;   // weak-form scratch [2N]
    const DenseOperator *dense = nullptr;   // assembled operator (FP32 form)
    int n64 = 0, n32 = 0;
    void apply(const double2 *v, double2 *out, int precision) {
        if (precision == BEM_FP32_DENSE) dense_gemv(*dense, v, yw, m->xs32, s);
        else farfield_apply(m, *nf, k0, k1, rho, v, yw, precision, s);
        osrc_apply_from_weak(m, *st, yw, out, s);
        if (precision == BEM_FP64) n64++;
        else n32++;
    }
};

struct Workspace {
    int64_t n2 = 0;
    int cap = 0;               // basis vectors beyond v_0
    DevBuf<double2> V;         // [cap + 1][n2]
    DevBuf<double2> h;         // [2 (cap + 1) + 1]
    void ensure(int need, hipStream_t s) {   // need = number of vectors
        if (need <= cap + 1) return;
        int ncap = std::max(need - 1, std::max(2 * cap, 64));
        DevBuf<double2> nv((size_t)(ncap + 1) * n2);
        if (V.p) BEM_HIP(hipMemcpyAsync(nv.p, V.p, (size_t)(cap + 1) * n2 * sizeof(double2),
                                        hipMemcpyDeviceToDevice, s));
        BEM_HIP(hipStreamSynchronize(s));
        V = std::move(nv);
        h.alloc(2 * (size_t)(ncap + 1) + 1);
        cap = ncap;
    }
};

double dev_norm(const double2 *v, int64_t n, double2 *hbuf, hipStream_t s) {
    blas_block_dot(v, n, 1, v, n, hbuf, s);
    double2 h;
    BEM_HIP(hipMemcpyAsync(&h, hbuf, sizeof(double2), hipMemcpyDeviceToHost, s));
    BEM_HIP(hipStreamSynchronize(s));
    if (!std::isfinite(h.x)) fail(BEM_E_NAN, "NaN/Inf in a vector norm");
    return std::sqrt(std::max(h.x, 0.0));
}

// Unrestarted GMRES on `op` (precision prec) for op(x) = b from x_0 = 0.
// Writes x; returns true when |g_{j+1}| <= tol ||b||.
bool gmres(Op &op, int prec, const double2 *b, double2 *x, int64_t n2, double tol,
           int maxiter, Workspace &ws, int &iters, double &est, hipStream_t s) {
    iters = 0;
    est = 0.0;
    ws.n2 = n2;
    ws.ensure(2, s);
    BEM_HIP(hipMemsetAsync(x, 0, n2 * sizeof(double2), s));
    const double beta = dev_norm(b, n2, ws.h.p, s);
    if (beta == 0.0) return true;
    if (maxiter < 1) return false;
    blas_axpby(make_double2(1.0 / beta, 0.0), b, make_double2(0, 0), nullptr, ws.V.p, n2, s);
    std::vector<cdd> H, cs, sn, g(1, cdd(beta));
    std::vector<double2> hh;
    int m = 0;
    bool conv = false;
    for (int j = 0; j < maxiter; j++) {
        ws.ensure(j + 2, s);
        double2 *Vj = ws.V.p + (size_t)j * n2, *Vn = ws.V.p + (size_t)(j + 1) * n2;
        op.apply(Vj, Vn, prec);
        double2 *h1 = ws.h.p, *h2 = ws.h.p + (j + 1), *nr = ws.h.p + 2 * (j + 1);
        blas_block_dot(ws.V.p, n2, j + 1, Vn, n2, h1, s);
        blas_block_axpy(ws.V.p, n2, h1, j + 1, -1.0, Vn, n2, s);
        blas_block_dot(ws.V.p, n2, j + 1, Vn, n2, h2, s);
        blas_block_axpy(ws.V.p, n2, h2, j + 1, -1.0, Vn, n2, s);
        blas_block_dot(Vn, n2, 1, Vn, n2, nr, s);
        blas_normalize(Vn, nr, n2, s);
        hh.resize(2 * (j + 1) + 1);
        BEM_HIP(hipMemcpyAsync(hh.data(), ws.h.p, hh.size() * sizeof(double2),
                               hipMemcpyDeviceToHost, s));
        BEM_HIP(hipStreamSynchronize(s));
        // column j of the Hessenberg matrix (stored by columns, length j + 2)
        std::vector<cdd> col(j + 2);
        for (int i = 0; i <= j; i++)
            col[i] = cdd(hh[i].x + hh[j + 1 + i].x, hh[i].y + hh[j + 1 + i].y);
        const double hn = std::sqrt(std::max(hh[2 * (j + 1)].x, 0.0));
        if (!std::isfinite(hn)) fail(BEM_E_NAN, "NaN/Inf in the Arnoldi process");
        col[j + 1] = hn;
        for (int i = 0; i < j; i++) {   // previous rotations
            cdd a = col[i], c = col[i + 1];
            col[i] = std::conj(cs[i]) * a + std::conj(sn[i]) * c;
            col[i + 1] = -sn[i] * a + cs[i] * c;
        }
        const double d = std::sqrt(std::norm(col[j]) + std::norm(col[j + 1]));
        cdd c0 = d > 0 ? col[j] / d : cdd(1.0), s0 = d > 0 ? col[j + 1] / d : cdd(0.0);
        cs.push_back(c0);
        sn.push_back(s0);
        col[j] = std::conj(c0) * col[j] + std::conj(s0) * col[j + 1];
        col[j + 1] = 0.0;
        g.push_back(-s0 * g[j]);
        g[j] = std::conj(c0) * g[j];
        H.insert(H.end(), col.begin(), col.begin() + (j + 1));   // R column j (rows 0..j)
        m = j + 1;
        est = std::abs(g[j + 1]) / beta;
        if (!std::isfinite(est)) fail(BEM_E_NAN, "NaN/Inf in the GMRES residual");
        if (est <= tol) {
            conv = true;
            break;
        }
    }
    iters = m;
    // back substitution R y = g (R upper triangular, columns stored packed)
    std::vector<cdd> y(m);
    auto R = [&](int i, int jj) { return H[(size_t)jj * (jj + 1) / 2 + i]; };
    for (int i = m - 1; i >= 0; i--) {
        cdd acc = g[i];
        for (int jj = i + 1; jj < m; jj++) acc -= R(i, jj) * y[jj];
        y[i] = acc / R(i, i);
    }
    std::vector<double2> yd(m);
    for (int i = 0; i < m; i++) yd[i] = make_double2(y[i].real(), y[i].imag());
    BEM_HIP(hipMemcpyAsync(ws.h.p, yd.data(), m * sizeof(double2), hipMemcpyHostToDevice, s));
    blas_block_axpy(ws.V.p, n2, ws.h.p, m, 1.0, x, n2, s);
    BEM_HIP(hipStreamSynchronize(s));
    return conv;
}

double2 damped(double2 k, double R) {
    // k_eps = k (1 + 0.4 i (k R)^{-2/3}), principal branch (Sec. 2.6)
    cdd kk(k.x, k.y);
    cdd ke = kk * (1.0 + cdd(0, 0.4) * std::pow(kk * R, -2.0 / 3.0));
    return make_double2(ke.real(), ke.imag());
}

// Krylov basis capacity after growing to `need` vectors (Workspace::ensure).
int64_t workspace_peak_vectors(int maxiter) {
    int cap = 0;
    int64_t peak = 0;
    auto ensure = [&](int need) {
        if (need <= cap + 1) return;
        const int ncap = std::max(need - 1, std::max(2 * cap, 64));
        peak = std::max<int64_t>(peak, (int64_t)(cap + 1) + (ncap + 1));   // old + new
        cap = ncap;
    };
    ensure(2);
    ensure(maxiter + 1);
    return std::max<int64_t>(peak, cap + 1);
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
    if (o.path < 0 || o.path > 2) fail(BEM_E_INVAL, "path must be 0, 1 or 2");
    for (int w = 0; w < n_waves; w++) {
        const double *d = dirs + 3 * w;
        if (!(std::fabs(std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) - 1.0) < 1e-6))
            fail(BEM_E_INVAL, "directions must be unit vectors");
    }
}

int64_t solve_footprint(bem_mesh *m, double2 k0, double2 k1, double rho,
                        const bem_solve_opts &o, int n_waves) {
    (void)rho;
    const int64_t n2 = 2 * m->N, c16 = (int64_t)sizeof(double2);
    int64_t b = 4 * m->nf_nnz * c16;                          // near-field CSR values
    b += osrc_state_bytes(m, o.pade_terms);                    // OSRC factors
    int64_t scratch = farfield_scratch_bytes(m, BEM_FP64, k0, k1);
    const bool dense = o.precision == BEM_FP32 && o.path == 1;
    if (o.precision == BEM_FP32 && !dense)
        scratch = std::max(scratch, farfield_scratch_bytes(m, BEM_FP32, k0, k1)) +
                  m->T * DYN_STRIDE * 4;                      // dyn32 beside dyn64
    b += scratch;
    if (dense) b += dense_bytes(m) + dense_assembly_scratch_bytes(m);
    b += ((int64_t)n_waves + 5) * n2 * c16;                    // f, yw, b, x, r, dx
    b += workspace_peak_vectors(o.maxiter) * n2 * c16 + (2 * (int64_t)o.maxiter + 8) * c16;
    return b;
}

int solve_run(bem_mesh *m, double2 k0, double2 k1, double rho, const double *directions,
              int n_waves, double tol, const bem_solve_opts &o, double2 *solution,
              bem_solve_info *info, hipStream_t s) {
    solve_check(m, k0, k1, rho, directions, n_waves, tol, o);
    if (!solution) fail(BEM_E_INVAL, "solution is NULL");
    const int64_t n2 = 2 * m->N;
    const NearOperator &nf = nearfield_get(m, k0, k1, rho, s);
    const double2 ko = o.osrc_interior ? k1 : k0;
    std::vector<double2> keps(m->nobj);
    for (int ob = 0; ob < m->nobj; ob++)
        keps[ob] = damped(ko, o.R > 0 ? o.R : 0.1 * m->obj_radius[ob]);
    OsrcState &st = osrc_get(m, o.pade_terms, o.theta, ko, keps, s);

    DevBuf<double2> f((size_t)n_waves * n2), yw(n2), b(n2), x(n2), r(n2), dx(n2);
    rhs_project(m, k0, directions, n_waves, f.p, s);
    Op op{m, &nf, k0, k1, rho, &st, s, yw.p};
    int inner = BEM_FP32;
    if (o.precision == BEM_FP32 && o.path != 0) {
        bool use = o.path == 1;
        if (o.path == 2) {   // dense when it fits with room to spare
            size_t free_b = 0, total_b = 0;
            BEM_HIP(hipMemGetInfo(&free_b, &total_b));
            use = dense_bytes(m) + (int64_t)(2ll << 30) < (int64_t)free_b ||
                  !m->dense_cache.empty();
        }
        if (use) {
            op.dense = &dense_get(m, k0, k1, rho, s);
            inner = BEM_FP32_DENSE;
        }
    }
    Workspace ws;
    ws.n2 = n2;
    ws.ensure(2, s);
    int worst = BEM_OK;
    for (int w = 0; w < n_waves; w++) {
        auto t0 = std::chrono::steady_clock::now();
        op.n64 = op.n32 = 0;
        osrc_apply_from_weak(m, st, f.p + (size_t)w * n2, b.p, s);
        const double bn = dev_norm(b.p, n2, ws.h.p, s);
        int total_it = 0, outer = 0;
        double rel = 0.0;
        bool conv = false;
        if (o.precision == BEM_FP64) {
            int it;
            double est;
            conv = gmres(op, BEM_FP64, b.p, x.p, n2, tol, o.maxiter, ws, it, est, s);
            total_it = it;
            outer = 1;
            op.apply(x.p, r.p, BEM_FP64);   // true residual with the FP64 operator
            blas_axpby(make_double2(1, 0), b.p, make_double2(-1, 0), r.p, r.p, n2, s);
            rel = bn > 0 ? dev_norm(r.p, n2, ws.h.p, s) / bn : 0.0;
        } else {
            BEM_HIP(hipMemsetAsync(x.p, 0, n2 * sizeof(double2), s));
            BEM_HIP(hipMemcpyAsync(r.p, b.p, n2 * sizeof(double2), hipMemcpyDeviceToDevice, s));
            double rn = bn;
            rel = bn > 0 ? 1.0 : 0.0;
            while (rel > tol && outer < o.max_outer && total_it < o.maxiter) {
                const double eta = std::min(0.5, o.inner_tol * tol * bn / rn);
                int it;
                double est;
                gmres(op, inner, r.p, dx.p, n2, eta, o.maxiter - total_it, ws, it, est, s);
                total_it += it;
                outer++;
                blas_axpby(make_double2(1, 0), x.p, make_double2(1, 0), dx.p, x.p, n2, s);
                op.apply(x.p, r.p, BEM_FP64);
                blas_axpby(make_double2(1, 0), b.p, make_double2(-1, 0), r.p, r.p, n2, s);
                rn = dev_norm(r.p, n2, ws.h.p, s);
                rel = rn / bn;
            }
            conv = rel <= tol;
        }
        BEM_HIP(hipMemcpyAsync(solution + (size_t)w * n2, x.p, n2 * sizeof(double2),
                               hipMemcpyDeviceToDevice, s));
        BEM_HIP(hipStreamSynchronize(s));
        const double secs =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (info) {
            info[w].iterations = total_it;
            info[w].outer_steps = outer;
            info[w].fp64_matvecs = op.n64;
            info[w].fp32_matvecs = op.n32;
            info[w].rel_residual = rel;
            info[w].seconds = secs;
        }
        if (!conv && rel > tol) worst = BEM_W_NOT_CONVERGED;
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
    o->inner_tol = 0.3;
    o->max_outer = 8;
    o->path = 2;
}

int pmchwt_solve(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int, double rho,
                 const double *directions, int n_waves, double tol,
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
                              (double2 *)solution, info, (hipStream_t)hip_stream);
    } catch (const bem::Error &e) {
        bem::set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        bem::set_last_error("host allocation failed");
        return BEM_E_NOMEM;
    }
}

}   // extern "C"

/*
 * bem.h -- C ABI of the MI355X (gfx950) OSRC-preconditioned PMCHWT library.
 *
 * Method: van 't Wout, Haqshenas, Gelat, Betcke, Saffari, "Frequency-robust
 * preconditioning of boundary integral equations for acoustic transmission",
 * J. Comput. Phys. 2022.  Section numbers below refer to that paper.
 *
 * Conventions shared by every call:
 *   - Return value: 0 = BEM_OK, > 0 warning, < 0 error; after an error the
 *     calling thread's message is available from bem_last_error().
 *   - bem_c64 has the layout of C99 double _Complex (torch.complex128).
 *   - Vectors x, y, solution are CALLER-OWNED DEVICE pointers on the current
 *     HIP device, row-major [n_rhs][2N] with each row = [psi (N); phi (N)]:
 *     psi = exterior Neumann trace, phi = Dirichlet trace of the total field
 *     (Sec. 2.2, unique pair of traces), P1 coefficients per vertex.  They must
 *     not alias; outputs are overwritten.
 *   - Work is enqueued on hip_stream (NULL = the null stream) and is
 *     stream-ordered; calls that return host data synchronise that stream.
 *   - A mesh handle owns all device state derived from the mesh (geometry,
 *     near-field operators, OSRC factors) and the device scratch its calls
 *     use.  Calls on one handle are stream-ordered; calls on the same handle
 *     from different streams or host threads must not overlap (they share
 *     that scratch).  Different handles are independent.  Creation and
 *     destruction are not thread-safe.
 */
#ifndef BEM_H
#define BEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } bem_c64;
typedef struct bem_mesh bem_mesh;

enum {
    BEM_OK = 0,
    BEM_W_NOT_CONVERGED = 1,   /* best iterate written */
    BEM_W_PENDING = 2,         /* bem_server_wait: not completed yet */
    BEM_W_DEFAULT = 3,         /* bem_tune_lookup: no tuned entry, defaults returned */
    BEM_E_INVAL = -1,          /* bad argument */
    BEM_E_BAD_MESH = -2,       /* not a closed, oriented, manifold surface */
    BEM_E_NOMEM = -3,          /* device allocation / budget exceeded */
    BEM_E_DEVICE = -4,         /* HIP runtime error */
    BEM_E_NAN = -5,            /* NaN/Inf in an iterate or residual */
    BEM_E_UNSUPPORTED = -6
};

/* Precision/path of the separated-pair part of the operator.  The singular
 * near field, OSRC and GMRES always run in FP64.
 *   BEM_FP64        matrix-free pair kernel in FP64
 *   BEM_FP32        matrix-free pair kernel in FP32
 *   BEM_FP32_DENSE  assembled dense complex64 operator [2N][2N] (FP32 pair
 *                   sums plus the FP64 near field rounded once), built on
 *                   first use for a (k_ext, k_int, rho) and kept resident;
 *                   needs 16 N^2 bytes of device memory (BEM_E_NOMEM else)
 *   BEM_FP64_DENSE  assembled dense complex128 operator (FP64 pair sums, the
 *                   FP64 pair kernel's quadrature and arithmetic), kept apart
 *                   from the complex64 one; 32 N^2 bytes.  One pass over it
 *                   per vector.
 *   BEM_FP32_HMAT   hierarchical form of the far part (the paper's operator
 *                   compression, Sec. 3.1): vertex cluster tree, admissible
 *                   cluster pairs (max diam <= eta dist) as adaptive cross
 *                   approximations U V^T to the relative tolerance tol,
 *                   other leaf pairs dense, entries as BEM_FP32_DENSE (FP32),
 *                   the FP64 near-field operator added; built on first use per
 *                   (k_ext, k_int, rho) and kept with the handle (two at
 *                   most); parameters from the tuning keys "hmat.*"; see
 *                   bem_hmat_info for its size.  Error against the exact
 *                   operator of the order of tol. */

enum { BEM_FP64 = 0, BEM_FP32 = 1, BEM_FP32_DENSE = 2, BEM_FP64_DENSE = 3, BEM_FP32_HMAT = 4 };

/*
 * Create the device state of a triangle surface mesh (Sec. 2.1: bounded
 * objects Omega_m with boundaries Gamma_m, outward unit normals; Sec. 2.3:
 * P1 elements on a triangular mesh).
 *   vertices   host, float64 [n_vertices][3]
 *   triangles  host, int32 [n_triangles][3], 0-based, counter-clockwise seen
 *              from outside ((v1-v0)x(v2-v0) points outward)
 *   object_id  host, int32 [n_triangles] in 0..n_objects-1, or NULL for one
 *              object; the vertices of each object must be contiguous
 * The inputs are copied; the caller keeps ownership.  Errors: BEM_E_INVAL
 * (sizes, indices out of range), BEM_E_BAD_MESH (degenerate triangle, edge
 * not shared by exactly two triangles with opposite orientation, object
 * with non-positive signed volume, vertex shared by two objects),
 * BEM_E_NOMEM, BEM_E_DEVICE.
 */
int bem_mesh_create(const double *vertices, int64_t n_vertices,
                    const int32_t *triangles, int64_t n_triangles,
                    const int32_t *object_id, bem_mesh **out);
void bem_mesh_destroy(bem_mesh *mesh);

/* Sizes of a mesh (any pointer may be NULL). */
int bem_mesh_info(const bem_mesh *mesh, int64_t *n_vertices,
                  int64_t *n_triangles, int32_t *n_objects,
                  int64_t *device_bytes);

/*
 * y = B x: the Galerkin (weak-form) permuted PMCHWT operator (Sec. 2.7,
 * single scatterer; multiple scatterers: exterior operators couple all
 * objects, interior ones act within each object)
 *     B = [[ V_0 + rho V_1 , -(K_0 + K_1)      ],
 *          [ K'_0 + K'_1   ,  D_0 + D_1 / rho  ]],
 * V, K, K' (the paper's T) and the Maue-form hypersingular D of Sec. 2.2 at
 * k_ext (index 0) and k_int (index 1), P1 test and trial functions (Sec. 2.3),
 * rho = rho_int / rho_ext.  Quadrature: 6-point rule per triangle for every
 * pair not sharing a vertex; Sauter-Schwab-type rules (4 Gauss points per
 * dimension) for coinciding, edge- and vertex-adjacent pairs.
 *   x, y       device, bem_c64 [n_rhs][2N]
 *   precision  BEM_FP64, BEM_FP32, BEM_FP32_DENSE or BEM_FP64_DENSE (see above)
 * The first call for a (k_ext, k_int, rho) builds and caches the near-field
 * operator on the device.  Errors: BEM_E_INVAL (rho <= 0, Im k < 0, k == 0,
 * n_rhs < 1, NULL pointers), BEM_E_NOMEM, BEM_E_DEVICE.
 */
int pmchwt_matvec(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int,
                  double rho, const bem_c64 *x, bem_c64 *y, int n_rhs,
                  int precision, void *hip_stream);

/*
 * pmchwt_matvec for objects of different materials (Sec. 2.7, multiple
 * scatterers; the paper's four-sphere test mixes two materials): object m
 * has interior wavenumber k_int[m] and density ratio rho[m] =
 * rho_int,m / rho_ext, so its interior operators are V_m, K_m, K'_m, D_m at
 * k_int[m], weighted by rho[m] and 1/rho[m]; the exterior operators couple
 * all objects as before.
 *   k_int, rho  host arrays [n_objects];  x, y as for pmchwt_matvec
 * The near-field and assembled operators are cached per set of materials.
 * Errors: as pmchwt_matvec, for every k_int[m] and rho[m].
 */
int pmchwt_matvec_multi(const bem_mesh *mesh, bem_c64 k_ext, const bem_c64 *k_int,
                        const double *rho, const bem_c64 *x, bem_c64 *y, int n_rhs,
                        int precision, void *hip_stream);

/*
 * y = B_M x: the Galerkin Mueller operator I + A_0 - A^_1 (Sec. 2.2; every
 * interface m contributes I_m + A_{0,mm} - A^_m, exterior operators A_{0,mn}
 * couple the objects) on the permuted unknowns x = [psi; phi] of
 * pmchwt_matvec:
 *     B_M = [[ V_0 - rho V_1  ,  M - (K_0 - K_1)   ],
 *            [ M + K'_0 - K'_1,  D_0 - D_1 / rho   ]],
 * M the P1 mass matrix (the identity tested against P1 functions, paired
 * with each trace row's own trace, hence off the diagonal after the
 * permutation).  Same quadrature, layouts, precisions and errors as
 * pmchwt_matvec; its near-field operator is cached apart from PMCHWT's.
 *   x, y  device, bem_c64 [n_rhs][2N]
 */
int muller_matvec(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int,
                  double rho, const bem_c64 *x, bem_c64 *y, int n_rhs,
                  int precision, void *hip_stream);

/*
 * y = diag(L_DtN, L_NtD) x in strong form (coefficients to coefficients),
 * the OSRC operators of Sec. 2.6 with damped wavenumber k_eps, square root
 * localised by an N_p-term Pade series with branch-cut rotation theta
 * (Sec. 2.7):  L_DtN = ik R(X),  L_NtD = (1/ik) R(X)(I + X)^{-1},
 * X = -M^{-1} S / k_eps^2 (P1 mass M, Laplace-Beltrami stiffness S),
 * R(z) = C_0 + sum_j A_j z / (1 + B_j z).  k and k_eps apply to every object.
 * The shifted sparse systems are factorised once per (k_eps, N_p, theta) and
 * cached on the device.
 *   x, y  device, bem_c64 [n_rhs][2N]
 * Errors: BEM_E_INVAL (pade_terms < 1 or > 32, k == 0, k_eps == 0).
 */
int osrc_apply(const bem_mesh *mesh, int pade_terms, double theta,
               bem_c64 k, bem_c64 k_eps, const bem_c64 *x, bem_c64 *y,
               int n_rhs, void *hip_stream);

/*
 * Sizes of the OSRC factors for (pade_terms, theta, k, k_eps) on this mesh
 * (created and cached as by osrc_apply when absent) and the algorithmic
 * device bytes of one single-vector osrc_apply (Sec. 2.7: N_p + 2 factorised
 * systems sharing one sparsity pattern; an apply makes 2 N_p + 2 block
 * solves, three P1 mass products and two Pade sums).  Each block solve
 * streams the entries of L outside the diagonal dissection blocks by rows and
 * by columns (16-byte values, 4-byte indices), the inverses of the diagonal
 * blocks of L and L^T, D^{-1}, and reads and writes one vector.
 * Errors: as osrc_apply; BEM_E_INVAL if out is NULL.
 */
typedef struct {
    int64_t n_vertices;
    int32_t pade_terms;
    int32_t n_factors;        /* pade_terms + 2 */
    int32_t solves_per_apply; /* 2 pade_terms + 2 */
    int32_t reserved0;
    int64_t nnz_l;            /* strict lower entries of L (one factor) */
    int64_t nnz_offblock;     /* of those, outside the diagonal dissection blocks */
    int64_t dense_entries;    /* entries of the dense diagonal-block inverses (one factor) */
    int64_t mass_nnz;         /* entries of the P1 mass matrix */
    int64_t factor_bytes;     /* device bytes of all numeric factors */
    int64_t bytes_per_apply;  /* algorithmic bytes of one single-vector apply */
} bem_osrc_stats;
int bem_osrc_info(const bem_mesh *mesh, int pade_terms, double theta,
                  bem_c64 k, bem_c64 k_eps, bem_osrc_stats *out,
                  void *hip_stream);

/*
 * osrc_apply without device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same operation, arguments, layouts and results as osrc_apply.
 *   - The OSRC factors for (pade_terms, theta, k, k_eps) must already be
 *     resident on the mesh handle (an earlier osrc_apply, or pmchwt_solve
 *     with those values, created them); otherwise BEM_E_INVAL and nothing is
 *     done.
 *   - The work vectors of the sweeps live in a library-owned device array of
 *     BEM_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends:
 *     min(n_rhs, 16) * ((2 pade_terms + 2) (3 n_vertices + P) +
 *     2 n_vertices) * 16 bytes must fit for pade_terms <= 16 (for more
 *     terms, whose solves run in two stages, (pade_terms + 2) (2 n_vertices
 *     + P) + (pade_terms + 5) n_vertices per vector; BEM_E_INVAL otherwise),
 *     P the partial sums of the top rows of the two-part block solve when
 *     the mesh's OSRC state has one ("osrc.split" = 2; a few thousand at
 *     10 242 vertices, else 0), e.g. 8 vectors of 10 242 vertices with 4
 *     Pade terms.  Nothing in it needs to start at zero.
 *   - Every call on one GPU uses that GPU's array: calls that overlap in time
 *     on one GPU (other streams, other threads) race; the caller serialises
 *     them.
 *   - No hipMalloc, hipFree or HIP event is made (profiling records nothing).
 */
#define BEM_NOALLOC_SCRATCH_BYTES (64ull << 20)
int osrc_apply_noalloc(const bem_mesh *mesh, int pade_terms, double theta,
                       bem_c64 k, bem_c64 k_eps, const bem_c64 *x, bem_c64 *y,
                       int n_rhs, void *hip_stream);

/*
 * Weak right-hand side [f_D; f_N] of the PMCHWT system for unit-amplitude
 * plane waves u_inc = exp(i k_ext d.x) (Sec. 2.1, Sec. 2.7):
 * f_D,i = int u_inc phi_i, f_N,i = int i k_ext (d.n) u_inc phi_i, 6-point rule.
 *   directions  host, float64 [n_waves][3] (unit vectors)
 *   f           device, bem_c64 [n_waves][2N]
 */
int pmchwt_rhs(const bem_mesh *mesh, bem_c64 k_ext, const double *directions,
               int n_waves, bem_c64 *f, void *hip_stream);

typedef struct {
    int pade_terms;      /* N_p, default 4 (Sec. 3.1) */
    double theta;        /* branch-cut rotation, default pi/3 */
    int osrc_interior;   /* 1: OSRC wavenumber k_int (default), 0: k_ext */
    double R;            /* k_eps radius; <= 0: 0.1 x object circumradius */
    int precision;       /* BEM_FP64 (plain GMRES) or BEM_FP32 (refinement) */
    int maxiter;         /* GMRES iterations cap (total), default 1000 */
    double inner_tol;    /* FP32 form: each inner GMRES stops at an absolute
                            residual inner_tol * tol * ||b|| (at most half of
                            the current outer residual); default 0.6 */
    int max_outer;       /* refinement steps cap, default 8 */
    int path;            /* operator of the GMRES iterations: 0 matrix-free
                            pair kernel, 1 assembled dense operator (complex64
                            for the FP32 form's inner solves, complex128 for
                            the FP64 form), 2 assembled when it fits in device
                            memory and, for the FP32 form, the autotuned table
                            does not prefer the matrix-free path (an assembly
                            that runs out of memory falls back to the
                            matrix-free operator) (default), 3 the compressed
                            operator (precision BEM_FP32 only: inner solves on
                            the H-matrix of bem_hmat_info, every outer
                            residual with the FP64 pair kernel) */
    int formulation;     /* BEM_FORM_OSRC (default), BEM_FORM_PMCHWT,
                            BEM_FORM_CALDERON or BEM_FORM_MULLER; see below */
} bem_solve_opts;

/* Formulations (the four compared in Sec. 3.1), all in strong form (mass
 * preconditioning, Sec. 2.4, M^{-1} on each N-block), f the weak right-hand
 * side, S the exchange of the two halves of a vector:
 *   BEM_FORM_OSRC      L M^{-1} B x = L M^{-1} f on x = [psi; phi],
 *                      L = diag(L_DtN, L_NtD) (OSRC, Sec. 2.6, 2.7)
 *   BEM_FORM_PMCHWT    M^{-1} B~ u = M^{-1} f, the standard PMCHWT on the
 *                      paper's ordering u = [phi; psi] (Sec. 2.2), B~ u = B x
 *   BEM_FORM_CALDERON  M^{-1} C M^{-1} B~ u = M^{-1} C M^{-1} f, C the
 *                      block-diagonal Calderon preconditioner (Sec. 2.5):
 *                      each object's own PMCHWT operator A_{0,mm} + A^_m
 *                      (with one object C = B~ in full; with several, C is
 *                      applied object by object through a mesh of each
 *                      object, built on first use and kept with the handle);
 *                      two operator applications per iteration.
 *   BEM_FORM_MULLER    M^{-1} B~_M u = M^{-1} f, the second-kind Mueller
 *                      formulation (Sec. 2.2, operator of muller_matvec)
 * OSRC, PMCHWT and Calderon solve the same discrete system B x = f; Mueller
 * is a different discretisation of the same problem.  GMRES always iterates
 * on x = [psi; phi] = S u; for the formulations on u it runs with the
 * operator conjugated by S, which leaves the residual history unchanged.
 * The solution is returned as x.  rel_residual and the tolerance refer to
 * the chosen preconditioned system. */
enum { BEM_FORM_OSRC = 0, BEM_FORM_PMCHWT = 1, BEM_FORM_CALDERON = 2, BEM_FORM_MULLER = 3 };

typedef struct {
    int iterations;      /* GMRES iterations (all inner solves) */
    int outer_steps;     /* refinement steps (1 for FP64) */
    int fp64_matvecs;
    int fp32_matvecs;
    double rel_residual; /* ||b - P x|| / ||b||, P with the FP64 operator; FP32
                            refinement with "solve.refine_update" = 1: an upper
                            bound, the FP64 residual of an earlier iterate
                            updated by FP32 products of the later corrections
                            plus the bound on their error */
    double seconds;      /* wall time of the solve of this wave's lockstep group, from
                            its first preconditioning to convergence; the set-up shared
                            by all waves (near field, OSRC factors, assembled operator)
                            is not included */
} bem_solve_info;

/* Fill *opts with the defaults above. */
void bem_solve_opts_default(bem_solve_opts *opts);

/*
 * Solve the OSRC-preconditioned permuted PMCHWT system (Sec. 2.7, strong
 * form Sec. 2.4) for each plane wave:
 *     L M^{-1} B x = L M^{-1} f,   L = diag(L_DtN, L_NtD) per object,
 * with unrestarted GMRES from x_0 = 0 (Sec. 3.1) to ||b - P x|| <= tol ||b||.
 * precision BEM_FP32: iterative refinement, outer residual with the FP64
 * operator (later ones updated with FP32 products of the corrections, see
 * "solve.refine_update"), inner GMRES on the operator with the FP32 pair
 * kernel, or on the assembled complex64 operator (path 1; see
 * "solve.residual_dense_gib" for how its FP64 residuals are formed), or on
 * the compressed operator (path 3; the H-matrix at the paper's ACA tolerance
 * 1e-5, Sec. 3.1), whose error the FP64 residuals of the outer steps remove.
 *   directions  host [n_waves][3];  solution  device [n_waves][2N]
 *   info        host [n_waves] or NULL
 * Returns BEM_W_NOT_CONVERGED (best iterate written) if maxiter is reached.
 * Errors: BEM_E_INVAL (bad options or directions; path 3 with precision
 * BEM_FP64), BEM_E_UNSUPPORTED (path 3 with the Calderon preconditioner of
 * several objects), BEM_E_NAN, BEM_E_NOMEM.
 */
int pmchwt_solve(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int,
                 double rho, const double *directions, int n_waves, double tol,
                 const bem_solve_opts *opts, bem_c64 *solution,
                 bem_solve_info *info, void *hip_stream);

/*
 * Total field at points off the surface from a solution x = [psi; phi] of
 * the plane wave u_inc = exp(i k_ext d.p), by the representation formulas
 * of Sec. 2.2 with the surface potentials of the total field:
 *   outside every object:  u(p) = u_inc(p) + sum over all triangles of
 *       int [ -G_0(p,y) psi(y) + (n_y . grad_y G_0(p,y)) phi(y) ] dy
 *   inside object m:       u(p) = int over object m's triangles of
 *       [ rho G_1(p,y) psi(y) - (n_y . grad_y G_1(p,y)) phi(y) ] dy
 * (G_m = e^{ik_m r}/(4 pi r); inside, the Neumann trace is rho times the
 * exterior one).  psi and phi are the P1 functions of the coefficients, the
 * 6-point rule per triangle is used, FP64 throughout.  The rule is that of
 * the matvec: accuracy drops for points closer to the surface than about
 * one triangle; points on the surface are not supported.  A point is inside
 * object m when the solid angle of m's surface at it (exact per flat
 * triangle) exceeds 2 pi in magnitude.
 *   direction  host float64 [3], unit;  solution  device bem_c64 [2N]
 *   points     device float64 [n_points][3];  out  device bem_c64 [n_points]
 *   region     device int32 [n_points] or NULL: 0 outside, m + 1 inside object m
 * n_points == 0 returns BEM_OK without touching the pointers.  Synchronises
 * the stream before returning.  Errors: BEM_E_INVAL (rho <= 0, bad k,
 * direction not unit, NULL pointers, n_points < 0).
 */
int pmchwt_field(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int, double rho,
                 const double *direction, const bem_c64 *solution, const double *points,
                 int64_t n_points, bem_c64 *out, int32_t *region, void *hip_stream);

/*
 * pmchwt_solve and pmchwt_field for objects of different materials (see
 * pmchwt_matvec_multi): k_int, rho host arrays [n_objects].  The OSRC
 * preconditioner of object m uses k_int[m] (osrc_interior) or k_ext, with
 * that object's damped wavenumber.
 */
int pmchwt_solve_multi(const bem_mesh *mesh, bem_c64 k_ext, const bem_c64 *k_int,
                       const double *rho, const double *directions, int n_waves, double tol,
                       const bem_solve_opts *opts, bem_c64 *solution, bem_solve_info *info,
                       void *hip_stream);
int pmchwt_field_multi(const bem_mesh *mesh, bem_c64 k_ext, const bem_c64 *k_int,
                       const double *rho, const double *direction, const bem_c64 *solution,
                       const double *points, int64_t n_points, bem_c64 *out, int32_t *region,
                       void *hip_stream);

/*
 * Far-field pattern F(xhat) of a solution: u_sca ~ F exp(i k r)/r with
 * F = 1/(4 pi) int exp(-i k xhat.y) [-psi - i k (xhat.n) phi] dy, from the
 * exterior representation formula (Sec. 2.2).
 *   solution device [2N];  dirs host [n_dirs][3];  out host [n_dirs]
 */
int bem_far_field(const bem_mesh *mesh, bem_c64 k_ext, const bem_c64 *solution,
                  const double *dirs, int n_dirs, bem_c64 *out,
                  void *hip_stream);

/*
 * Serving loop: a queue of solve requests run by a pool of worker threads,
 * each with its own HIP stream, so that the work of several requests overlaps
 * on the device.  Requests name a mesh registered with the server; each mesh
 * keeps up to max_replicas device-resident handles, whose near-field and OSRC
 * caches stay resident between requests; the handles of a mesh share its
 * assembled operators (one assembly per wavenumbers and materials, awaited by
 * a replica that needs one another replica is assembling; besides the ones
 * running requests use, the most recent one is kept).  A handle serves one
 * request at a time.
 *
 * Admission: a request starts when a worker and a handle of its mesh are free
 * and its device-memory footprint (an upper bound of what the solve
 * allocates: near field, OSRC factors, scratch, the initial Krylov basis of 65
 * vectors per wave, the dense operator on the assembled path) fits in the
 * budget beside the resident state of all handles and the footprints of
 * running requests.  A running request's Krylov basis doubles as it fills;
 * each growth is added to its reservation as it happens, releasing cached
 * state if needed, and runs on even when the budget is exceeded (at most
 * maxiter + 1 vectors per wave).  When a request does not fit, the caches of
 * idle handles are released, least recently used first.  Assembled
 * operators that no request holds stay resident outside the budget, as a
 * cache whose buffers new operators reuse; when a device allocation fails,
 * they are released first (least recently used), then the caches of idle
 * handles, and the allocation is retried.  A request that cannot fit even on an idle
 * server completes with status BEM_E_NOMEM.  Waiting requests are admitted
 * smallest estimated work first (triangle pairs of the assembly or of the
 * matrix-free products, operator entries read by the iterations), except that
 * requests that have waited 2 s go first in arrival order, and once the
 * oldest has waited 10 s no other request starts while it does not fit.
 *
 * Path: opts.path 2 (auto) becomes the assembled path when the dense
 * operator (complex64 for FP32, complex128 for FP64) is at most
 * dense_max_bytes and the autotuned table does not prefer the matrix-free
 * path, else matrix-free; the
 * choice depends only on the request, so a result does not depend on the
 * other requests in flight.
 */
typedef struct bem_server bem_server;

typedef struct {
    int64_t hbm_budget;      /* bytes; <= 0: 90 % of free device memory at creation */
    int workers;             /* concurrent requests (threads, streams); <= 0: 4; max 64 */
    int max_replicas;        /* handles per registered mesh; <= 0: workers */
    int64_t dense_max_bytes; /* auto path limit for the assembled operator; < 0: 16 GiB */
} bem_server_opts;

typedef struct {
    int status;              /* return code of the solve (BEM_OK, BEM_W_NOT_CONVERGED, < 0) */
    int path;                /* 0 matrix-free, 1 assembled, 3 compressed operator */
    double t_submit;         /* seconds since server creation */
    double t_admit;
    double t_end;
    int64_t footprint;       /* admission estimate, bytes */
    int replica;             /* handle index within its mesh */
} bem_request_stats;

typedef struct {
    int64_t budget;          /* bytes */
    int64_t resident_bytes;  /* cached state of all handles */
    int64_t reserved_bytes;  /* footprints of running requests */
    int64_t peak_bytes;      /* max over time of resident + reserved */
    int inflight, peak_inflight, queued;
    int64_t completed, rejected;
    int64_t evictions;       /* cached states released: idle handles' caches, and
                                assembled operators no request held (on a
                                failed device allocation) */
    int64_t krylov_growth_bytes; /* Krylov-basis growth reported by running
                                    requests beyond their footprints (total) */
} bem_server_stats;

void bem_server_opts_default(bem_server_opts *opts);
/* Create on the current device; opts NULL = defaults. */
int bem_server_create(const bem_server_opts *opts, bem_server **out);
/* Waits for running requests; requests still queued complete with
 * BEM_E_INVAL ("server shut down").  Handles of registered meshes are freed. */
void bem_server_destroy(bem_server *srv);
/* Register a mesh (same arguments and validation as bem_mesh_create); one
 * handle is created and its OSRC symbolic analysis run now. */
int bem_server_add_mesh(bem_server *srv, const double *vertices, int64_t n_vertices,
                        const int32_t *triangles, int64_t n_triangles,
                        const int32_t *object_id, int *mesh_id);
/* Queue one solve (arguments as pmchwt_solve).  solution: caller-owned
 * device [n_waves][2N]; info: caller-owned host [n_waves] or NULL; both must
 * stay valid until bem_server_wait returns for this request.  directions and
 * opts are copied.  Argument errors are returned here (nothing queued). */
int bem_server_submit(bem_server *srv, int mesh_id, bem_c64 k_ext, bem_c64 k_int, double rho,
                      const double *directions, int n_waves, double tol,
                      const bem_solve_opts *opts, bem_c64 *solution, bem_solve_info *info,
                      int64_t *request_id);
/* bem_server_submit for objects of different materials (see
 * pmchwt_matvec_multi): k_int, rho host arrays [n_objects], copied. */
int bem_server_submit_multi(bem_server *srv, int mesh_id, bem_c64 k_ext, const bem_c64 *k_int,
                            const double *rho, const double *directions, int n_waves, double tol,
                            const bem_solve_opts *opts, bem_c64 *solution, bem_solve_info *info,
                            int64_t *request_id);
/* Wait up to timeout_s seconds (< 0: forever).  Returns BEM_OK when the
 * request has completed (its status, timing and path in *stats; the request
 * is then forgotten), BEM_W_PENDING on time-out, BEM_E_INVAL for an unknown
 * id.  When the request's status is an error, bem_last_error() on the waiting
 * thread holds its message. */
int bem_server_wait(bem_server *srv, int64_t request_id, double timeout_s,
                    bem_request_stats *stats);
int bem_server_stats_get(bem_server *srv, bem_server_stats *stats);

/* Kernel timing with HIP events recorded on the launch stream, for the named
 * kernel ("farfield_fp32", "farfield_fp64", "nearfield_spmv", ...).
 * enable = 1 starts recording (and resets), 0 stops.  bem_profile_read
 * synchronises the recorded events and returns total milliseconds and the
 * launch count since the last reset. */
int bem_profile_enable(int enable);
int bem_profile_read(const char *kernel, double *total_ms, int64_t *launches);

/* Process-wide default launch parameters, used for shapes without an
 * autotuned entry:
 *   "farfield.multi_max"  right-hand sides sharing one pair-kernel launch on
 *                         the FP32 matrix-free path: 1, 2 or 4 (default 4)
 *   "farfield.block"      test triangles per pair-kernel workgroup: 64, 128
 *                         or 256 (default 256)
 *   "farfield.symmetric"  1: a single FP32 right-hand side evaluates every
 *                         separated triangle pair once and adds it to the
 *                         rows of both triangles (the kernels of V, K, K'
 *                         and D in Maue form depend on the points only
 *                         through r; Sec. 2.2); 0: each ordered pair in the
 *                         one-directional kernel (default 1)
 *   "farfield.sym_round_mib" symmetric kernel: largest buffer of the partial
 *                         sums of the second triangle's rows per launch, in
 *                         MiB (1..65536, default 4096: one launch up to about
 *                         60 000 vertices); larger meshes run the test blocks
 *                         in several launches, results unchanged
 *   "dense.skinny_min_rhs" right-hand-side count (>= 2) from which products
 *                         with the assembled operator below gemm_min use the
 *                         16-column MFMA kernel instead of the multi-vector
 *                         GEMV (default 24: not below the default gemm_min)
 *   "dense.gemm_min_rhs"  right-hand-side count from which the assembled
 *                         operator is applied with the MFMA product instead of
 *                         the multi-vector product, 8 vectors per pass
 *                         (default 24)
 *   "solve.refine_update" FP32 refinement (precision BEM_FP32 in
 *                         pmchwt_solve): 1 forms the first outer residual
 *                         b - P64 x with the FP64 operator and updates the
 *                         later ones as r - P32 d, the FP32 product of the
 *                         small correction d, carrying the bound 1e-4 |P32 d|
 *                         of that product's error into the reported residual
 *                         (formed in FP64 again before the carried bound
 *                         reaches tol / 10); 0 forms every outer residual with
 *                         the FP64 operator (default 1)
 *   "solve.residual_dense_gib" assembled FP32 path (path 1, precision
 *                         BEM_FP32): when the complex128 operator is at most
 *                         this many GiB, the operator is assembled once in
 *                         FP64, the inner solves use its rounding to
 *                         complex64 and the FP64 residuals the complex128
 *                         operator; else the complex64 operator is assembled
 *                         in FP32 and the FP64 residuals are matrix-free.
 *                         0..1024, 0 disables (default 32)
 *   "hmat.leaf"           compressed operator: vertices per leaf cluster,
 *                         8..64 (default 64)
 *   "hmat.eta_pct"        admissibility parameter eta in percent (default
 *                         100: max diameter <= distance)
 *   "hmat.tol_ppb"        ACA tolerance in parts per 1e9 (default 10000 =
 *                         1e-5, the paper's)
 *   "hmat.kmax"           largest rank of a block, 4..512 (default 128)
 *   "osrc.split"          OSRC block solves (keys read when a mesh handle
 *                         first builds its OSRC state): 1 (default) solves
 *                         the bottom subtrees of the nested dissection in
 *                         one workgroup each (rows in LDS), then the top
 *                         separators one launch per dissection level (two
 *                         for the levels of few, large blocks); plans with
 *                         subtrees of up to 512, 1024, 2048 and 4096 rows,
 *                         each batch taking subtrees of up to 2048 rows, or
 *                         larger ones when they still give 1024 workgroups
 *                         (subtrees x systems x vectors); 0 one launch per
 *                         level throughout; 2 the two-part solve whose
 *                         subtree workgroups also form the top rows' partial
 *                         sums, the top part in one workgroup when small; 3
 *                         as 1 with the one plan of "osrc.bottom_rows"
 *   "osrc.sub_rows"       largest subtree of "osrc.split" 2 in rows,
 *                         64..8192, 0 for 4096 or the device's LDS limit
 *                         (default 0)
 *   "osrc.top_single_work" "osrc.split" 2: top part in one workgroup when
 *                         its entries (L and dense block inverses) are at
 *                         most this many, else level by level (default 300000)
 *   "osrc.bottom_rows"    largest subtree of "osrc.split" 3 in rows, 64..8192
 *                         (default 1024)
 * Results of a solve depend on these (the summation order changes), within
 * the FP32 accuracy; with "osrc.split" = 1 an OSRC apply's rounding also
 * depends on the batch size and the number of Pade terms.  BEM_E_INVAL for an unknown key or value. */
int bem_tune_set(const char *key, int64_t value);
int bem_tune_get(const char *key, int64_t *value);

/* Size and set-up cost of the compressed operator (BEM_FP32_HMAT) of a
 * wavenumber pair; builds it if needed. */
typedef struct {
    int64_t bytes;            /* device bytes of the whole operator */
    int64_t lowrank_bytes;    /* U, V factors */
    int64_t dense_bytes;      /* dense leaf blocks */
    int32_t n_clusters, n_admissible, n_dense, max_rank;
    int32_t split_blocks;     /* admissible blocks split into their children after
                                 kmax terms above the tolerance */
    int32_t leaf, kmax;
    double mean_rank;
    double admissible_fraction;   /* share of the 4 N^2 entries in low-rank blocks */
    double eta, tol;
    double setup_seconds;     /* tree, ACA and dense blocks (wall clock) */
    double alpha;             /* scaling of the phi rows and columns during the
                                 cross approximation (balances the blocks) */
} bem_hmat_stats;
int bem_hmat_info(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int, double rho,
                  bem_hmat_stats *out, void *hip_stream);

/*
 * Autotuner.  For a mesh size (triangle count) and a right-hand-side count it
 * times, on the device, the pair-kernel workgroup size (64, 128 or 256 test
 * triangles) and the right-hand sides per launch (1, 2, 4) of the FP32
 * matrix-free operator, and, when the assembled complex64 operator fits in
 * free device memory with 2 GiB to spare, its assembly and the product with
 * n_rhs vectors (multi-vector GEMV, 16-column MFMA kernel or MFMA GEMM).  The
 * assembled path is chosen when assembly + expected_matvecs products beat
 * expected_matvecs matrix-free applications.  The result is kept for (n_triangles, bucket of n_rhs:
 * 1, 2-3, 4-7, 8-15, 16+) and used by every later matvec and solve of that
 * shape: launch parameters always, the path when opts.path is 2 (auto).
 * When a cache file was named with bem_tune_cache_load, new entries are
 * appended to it.  The timing input is zero vectors; the operator is built
 * for (k_ext, k_int, rho) and the assembled one freed after timing.
 */
typedef struct {
    int block;               /* test triangles per pair-kernel workgroup */
    int multi;               /* right-hand sides per pair-kernel launch */
    int gemm_min;            /* assembled path: MFMA GEMM from this many vectors */
    int skinny_min;          /* below gemm_min: 16-column MFMA product from this many, else
                                the multi-vector GEMV */
    int path;                /* -1 no preference, 0 matrix-free, 1 assembled */
    double t_matrix_free;    /* seconds per operator application to n_rhs vectors */
    double t_assembled;      /* same on the assembled operator (0 if not timed) */
    double t_assembly;       /* seconds to assemble (0 if not timed) */
} bem_tune_entry;

int bem_autotune(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int, double rho, int n_rhs,
                 int expected_matvecs, bem_tune_entry *out, void *hip_stream);
/* Load entries for `arch` (NULL: the current device's, e.g. "gfx950") from a
 * cache file and append later autotune results to it.  A missing file is an
 * empty cache.  Malformed lines and other architectures are skipped. */
int bem_tune_cache_load(const char *path, const char *arch, int *n_loaded);
/* Entry for a shape: BEM_OK if tuned, BEM_W_DEFAULT with the defaults if not. */
int bem_tune_lookup(int64_t n_triangles, int n_rhs, bem_tune_entry *out);
/* Forget all tuned entries and the cache file name. */
void bem_tune_clear(void);

/* Diagnostic for the issue-bound roofline of the pair kernel: measured issue
 * rates, in lane operations per second summed over the device, of
 * rates[0] v_fma_f32, [1] v_sin_f32, [2] v_cos_f32, [3] v_rsq_f32 and
 * [4] v_fma_f64.  Each comes from a micro-kernel with 8 independent
 * dependency chains per lane at full occupancy (about 10 ms in total).
 *   rates  host [5], written on success
 * Allocates and frees 4 MiB of device memory; synchronises the stream. */
int bem_valu_rates(double *rates, void *hip_stream);

/* Message of the last error on the calling thread ("" if none). */
const char *bem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BEM_H */

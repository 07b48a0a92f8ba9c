// Internal declarations of the PMCHWT/OSRC library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <atomic>
#include <condition_variable>
#include <map>
#include <mutex>
#include <set>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "bem.h"

namespace bem {

struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);
void set_last_error(const std::string &msg);

// Device memory pressure: when an allocation fails, the registered
// releasers (the serving loop's idle caches) are asked to free something;
// release_device_memory returns whether any did, and the allocation is
// retried.
using MemReleaser = bool (*)(void *ctx);
void add_mem_releaser(MemReleaser fn, void *ctx);
void remove_mem_releaser(void *ctx);
bool release_device_memory();

#define BEM_HIP(expr)                                                         \
    do {                                                                      \
        hipError_t e_ = (expr);                                               \
        if (e_ != hipSuccess)                                                 \
            ::bem::fail(BEM_E_DEVICE, std::string(#expr) + ": " +             \
                                          hipGetErrorString(e_));             \
    } while (0)

#define BEM_LAUNCH_CHECK() BEM_HIP(hipGetLastError())

// Owning device buffer.
template <class T> struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        hipError_t e = hipMalloc((void **)&p, count * sizeof(T));
        while (e == hipErrorOutOfMemory && release_device_memory()) {
            (void)hipGetLastError();
            e = hipMalloc((void **)&p, count * sizeof(T));
        }
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            fail(BEM_E_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) +
                                  " bytes failed: " + hipGetErrorString(e));
        }
        n = count;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void upload(const std::vector<T> &h) {
        if (h.size() != n) alloc(h.size());
        if (n) BEM_HIP(hipMemcpy(p, h.data(), n * sizeof(T), hipMemcpyHostToDevice));
    }
    size_t bytes() const { return n * sizeof(T); }
};

// ---------------------------------------------------------------- quadrature
struct Rules {
    double reg_bary[6][3];   // 6-point rule, barycentric (phi_0, phi_1, phi_2)
    double reg_w[6];         // weights, sum 1
    // singular rules over K x K, K = {0 <= x2 <= x1 <= 1}: rows x1 x2 y1 y2 w
    std::vector<double> ss[3];   // 0 coincident, 1 common edge, 2 common vertex
};
const Rules &rules();

// ------------------------------------------------------------- device layout
// Per-triangle static geometry record (FP64 and FP32 copies, the FP32 one in
// coordinates centred on the bounding-box centre):
//   [0..17]  the 6 quadrature points (x,y,z) of the 6-point rule
//   [18..20] unit normal n
//   [21]     plane offset c = n . v0  (n . p is the same for every p on it)
constexpr int GEO_STRIDE = 22;
// Per-triangle dynamic source record of one right-hand side:
//   [0..11]  s_psi(q_j) = w_j |sigma| sum_b phi_b(q_j) psi_b, complex, j=0..5
//   [12..23] s_phi(q_j), same with phi
//   [24..29] sC = |sigma| sum_b curl(phi_b) phi_b  (3 complex)
constexpr int DYN_STRIDE = 30;
// Test-side contraction data per triangle:
//   [0] |tau|   [1..9] curl phi_a (a-major, xyz)
constexpr int TST_STRIDE = 10;
// Partial far-field rows per (split, test triangle): 12 doubles
//   row1[a] (re,im) a=0..2, row2[a] (re,im) a=0..2
constexpr int ROW_STRIDE = 12;

// s1: sign of the interior operators, +1 PMCHWT, -1 Mueller (which also
// carries the identity term in its near field)
struct NearKey {
    double k0r, k0i, k1r, k1i, rho;
    int s1;
    std::vector<double> om;   // per object (Re k_m, Im k_m, rho_m) when they differ, else empty
    bool operator<(const NearKey &o) const {
        return std::tie(k0r, k0i, k1r, k1i, rho, s1, om) <
               std::tie(o.k0r, o.k0i, o.k1r, o.k1i, o.rho, o.s1, o.om);
    }
};

struct NearOperator {
    DevBuf<double> vals;   // [4 blocks][nnz] complex (interleaved): B11 B12 B21 B22
    int s1 = 1;            // operator the values belong to (NearKey::s1)
    // interior material of each object, and the wavenumber that decides the
    // pair kernels' variant (largest |Re k_m|; complex when any k_m is)
    std::vector<double2> k1o;
    std::vector<double> rhoo;
    double2 k1_plan{0.0, 0.0};
    // per-object interior coefficients of the pair kernels (several objects;
    // filled on first use)
    mutable DevBuf<float> itab32;
    mutable DevBuf<double> itab64;
};

// Interior materials of the objects when they differ (Sec. 2.7, several
// scatterers): k_m and rho_m = rho_int,m / rho_ext per object.
struct ObjMaterials {
    std::vector<double2> k;
    std::vector<double> rho;
};

// Assembled complex64 operator [2N][2N] (row-major).
struct DenseOperator {
    int64_t n2 = 0;
    int64_t T = 0;             // triangles of the mesh (tuning lookups)
    bool fp64 = false;         // B64 (complex128) instead of B (complex64)
    DevBuf<float2> B;
    DevBuf<double2> B64;
    // Split-K workspace of the MFMA product, kept between calls: a freshly
    // allocated one costs the product 5-10 % (first use of its pages).  One
    // call at a time holds it (until its kernels have finished); a concurrent
    // call on the same operator allocates its own.
    struct GemmWork {
        std::mutex mu;
        DevBuf<float> Xp, Yp;
        std::atomic<int64_t> held{0};
    };
    std::unique_ptr<GemmWork> gw = std::make_unique<GemmWork>();
    int64_t bytes() const { return B.bytes() + B64.bytes() + gw->held.load(); }
};

// Assembled operators: complex64 from the FP32 assembly, complex128 from the
// FP64 assembly, and complex64 rounded from the complex128 one (the assembled
// FP32 path when its FP64 residuals use the complex128 operator).
enum DenseKind { DENSE_C64 = 0, DENSE_C128 = 1, DENSE_C64_ROUNDED = 2 };

// Assembled operators shared by the handles (replicas) of one mesh in the
// serving loop: one assembly per (wavenumbers, materials, precision), reused
// by every replica; beyond `keep`, operators that no request holds are
// dropped, least recently used first.
struct DenseShare {
    using Key = std::pair<NearKey, int>;   // int: DenseKind
    struct Entry {
        std::shared_ptr<DenseOperator> op;
        uint64_t last = 0;
    };
    std::mutex mu;
    std::condition_variable cv;
    std::map<Key, Entry> ops;
    std::set<Key> building;   // assemblies in progress (other replicas wait)
    int keep = 2;   // e.g. a complex128 operator and its rounded complex64 one
    int64_t bytes();
    int64_t idle_bytes();   // operators no request holds (the others are in footprints)
    // Drops the least recently used operator that no request holds; returns
    // its bytes (0: none) and its last-use stamp through *last.
    int64_t evict_idle_lru();
    uint64_t oldest_idle();   // last-use stamp of that operator (UINT64_MAX: none)
};

struct OsrcKey {
    int np;
    double theta, kr, ki;
    std::vector<double> keps;   // (re, im) of k_eps per object
    std::vector<double> kobj;   // (re, im) of k per object when they differ, else empty
    bool operator<(const OsrcKey &o) const {
        return std::tie(np, theta, kr, ki, keps, kobj) <
               std::tie(o.np, o.theta, o.kr, o.ki, o.keps, o.kobj);
    }
};

struct OsrcState;   // defined in osrc.cpp
struct OsrcDeleter {
    void operator()(OsrcState *p) const;   // osrc.cpp
};
int64_t osrc_bytes(const OsrcState &st);
struct OsrcStats {
    int64_t n, nnz_l, nnz_ext, ndense, mass_nnz, factor_bytes, bytes_per_apply;
    int np, nfactors, solves;
};
OsrcStats osrc_stats(const bem_mesh *m, const OsrcState &st);
struct HMatrix;   // hmat.hip
struct HMatDeleter {
    void operator()(HMatrix *p) const;
};

struct OsrcSymbolicState;   // osrc.cpp
struct OsrcSymDeleter {
    void operator()(OsrcSymbolicState *p) const;
};
int64_t osrc_sym_bytes(const OsrcSymbolicState &st);

struct Profile;

}   // namespace bem

struct bem_mesh {
    int64_t N = 0, T = 0;
    int nobj = 1;
    std::vector<double> P;          // [N][3]
    std::vector<int32_t> tri;       // [T][3]
    std::vector<int32_t> tobj;      // [T]
    std::vector<int32_t> vobj;      // [N]
    std::vector<double> area;       // [T]
    std::vector<double> normal;     // [T][3]
    std::vector<double> curl;       // [T][3][3]
    double centre[3] = {0, 0, 0};
    double diameter = 0;            // bounding-box diagonal
    std::vector<double> obj_radius; // circumradius about each object's centroid

    // device geometry
    bem::DevBuf<double> geo64;      // [T][GEO_STRIDE]
    bem::DevBuf<float> geo32;       // [T][GEO_STRIDE]
    bem::DevBuf<double> tst;        // [T][TST_STRIDE]
    bem::DevBuf<int32_t> tobj_d;    // [T]
    bem::DevBuf<int32_t> tri_d;     // [T][3]
    bem::DevBuf<int32_t> star_ptr;  // [N+1] vertex -> (tri*3 + a), ascending
    bem::DevBuf<int32_t> star_idx;
    bem::DevBuf<double> P_d;        // [N][3] vertices (field evaluation; on first use)

    // near field: ordered pairs (tau, sigma) sharing >= 1 vertex
    int64_t n_near = 0;
    bem::DevBuf<int32_t> near_pairs;   // [n_near][4]: tau, sigma, class, perms
    bem::DevBuf<int32_t> nf_rowptr;    // [N+1]
    bem::DevBuf<int32_t> nf_col;       // [nnz]
    bem::DevBuf<int32_t> nf_cptr;      // [nnz+1]
    bem::DevBuf<int32_t> nf_contrib;   // pair*9 + a*3 + b
    int64_t nf_nnz = 0;
    bem::DevBuf<double> ss_tab;        // concatenated singular rules [n][5]
    int ss_off[4] = {0, 0, 0, 0};      // row offsets of the three rules
    std::map<bem::NearKey, std::unique_ptr<bem::NearOperator>> near_cache;
    std::map<bem::NearKey, std::unique_ptr<bem::DenseOperator>> dense_cache;
    std::map<bem::NearKey, std::unique_ptr<bem::DenseOperator>> dense64_cache;   // complex128
    std::map<bem::NearKey, std::unique_ptr<bem::DenseOperator>> dense_rounded_cache;   // of dense64
    std::map<bem::NearKey, std::unique_ptr<bem::HMatrix, bem::HMatDeleter>> hmat_cache;
    std::shared_ptr<bem::DenseShare> dense_share;   // set for serving replicas
    bem::DevBuf<float2> xs32;          // complex64 copy of a matvec input

    // OSRC: P1 vertex graph, M and S values, factor state per parameter set
    std::unique_ptr<bem::OsrcSymbolicState, bem::OsrcSymDeleter> osrc_sym;
    std::map<bem::OsrcKey, std::unique_ptr<bem::OsrcState, bem::OsrcDeleter>> osrc_cache;

    // scratch (grown on demand)
    bem::DevBuf<double> dyn64;
    bem::DevBuf<float> dyn32;
    bem::DevBuf<double> partial;
    bem::DevBuf<double> trirows;
    bem::DevBuf<int32_t> sym_items;      // work items of the symmetric pair kernel
    const void *sym_plan_id = nullptr;   // plan whose items sym_items holds

    // each object as a mesh of its own (block-diagonal Calderon
    // preconditioner; built on first use): part o holds object o's vertices
    // in ascending global order, part_vidx[o] their global ids
    std::vector<std::unique_ptr<bem_mesh>> parts;
    std::vector<bem::DevBuf<int32_t>> part_vidx;

    int64_t device_bytes() const;
    ~bem_mesh();
};

namespace bem {

// Process-wide default launch parameters (bem_tune_set / bem_tune_get).
struct Tuning {
    std::atomic<int> farfield_multi_max{4};   // right-hand sides per pair-kernel launch
    std::atomic<int> farfield_block{256};     // test triangles per pair-kernel workgroup
    std::atomic<int> farfield_symmetric{1};   // FP32 single vector: each separated pair once
    std::atomic<int> farfield_sym_round_mib{4096};   // symmetric kernel: sigma partials per launch
    std::atomic<int> dense_gemm_min_rhs{24};  // MFMA product from this many right-hand sides
    std::atomic<int> dense_skinny_min_rhs{24}; // skinny MFMA product from this many (else multi-GEMV)
    std::atomic<int> solve_refine_update{1};  // FP32 refinement: later residuals updated in FP32
    std::atomic<int> solve_residual_dense_gib{32};   // complex128 operator for FP32-path residuals
    // compressed operator (read when one is built)
    std::atomic<int> hmat_leaf{64};           // vertices per leaf cluster (<= 64)
    std::atomic<int> hmat_eta_pct{100};       // admissibility max(diam) <= eta dist, percent
    std::atomic<int64_t> hmat_tol_ppb{10000}; // ACA tolerance, parts per 1e9 (1e-5)
    std::atomic<int> hmat_kmax{128};          // largest rank of a block
    // OSRC block solves (read when a mesh's OSRC symbolic state is built)
    std::atomic<int> osrc_split{1};           // 0 levels, 1 bottom subtrees (plan per
                                              // batch), 2 two-part with partial sums,
                                              // 3 bottom subtrees of osrc_bottom_rows
    std::atomic<int> osrc_bottom_rows{1024};  // largest subtree of the bottom-subtree schedule
    std::atomic<int> osrc_sub_rows{0};        // largest bottom subtree (rows); 0: 4096 or the LDS limit
    std::atomic<int> osrc_top_single_work{300000};   // top part in one workgroup up to this work
};
Tuning &tuning();

// Launch parameters for one (triangle count, right-hand-side bucket): an
// autotuned entry (tune.cpp) or the defaults above.
struct TuneEntry {
    int block = 256;           // test triangles per pair-kernel workgroup: 64, 128, 256
    int multi = 4;             // right-hand sides per pair-kernel launch: 1, 2, 4
    int gemm_min = 24;         // MFMA product from this many right-hand sides
    int skinny_min = 24;       // below gemm_min: skinny MFMA product from this many, else multi-vector GEMV
    int path = -1;             // FP32 solves: -1 no preference, 0 matrix-free, 1 assembled
    double t_mf = 0, t_dense = 0, t_asm = 0;   // seconds (R vectors; assembly)
};
int tune_bucket(int R);                    // 1, 2, 4, 8 or 16
TuneEntry tune_lookup(int64_t T, int R);   // tuned entry, else defaults
bool tune_find(int64_t T, int R, TuneEntry *e);

// farfield.hip
void farfield_apply(bem_mesh *m, const NearOperator &nf, double2 k0, double2 k1,
                    double rho, const double2 *x, double2 *y, int precision,
                    hipStream_t s, int block = 0);
// y_r = B x_r for R right-hand sides ([R][2N]); FP32 shares each kernel
// evaluation among up to 4 right-hand sides
// Launch parameters: tune_lookup(T, R) unless `forced` is given.
void farfield_apply_batch(bem_mesh *m, const NearOperator &nf, double2 k0, double2 k1,
                          double rho, const double2 *x, double2 *y, int R, int precision,
                          hipStream_t s, const TuneEntry *forced = nullptr);
// device scratch (source records, split partials, triangle rows) that
// farfield_apply_batch needs for this precision, wavenumber pair and R
int64_t farfield_scratch_bytes(const bem_mesh *m, int precision, double2 k0, double2 k1, int R);
// nearfield.hip
// s1 = +1: near field of the permuted PMCHWT operator; s1 = -1: of the
// Mueller operator on the same unknowns (interior terms negated, P1 mass
// matrix added to the two off-diagonal blocks).  The pair kernels read s1
// from the near operator they are given.
// om: per-object materials (nullptr: every object has k1, rho).
std::unique_ptr<NearOperator> nearfield_build(bem_mesh *m, double2 k0, double2 k1,
                                              double rho, hipStream_t s, int s1,
                                              const ObjMaterials *om = nullptr);
const NearOperator &nearfield_get(bem_mesh *m, double2 k0, double2 k1, double rho,
                                  hipStream_t s, int s1 = 1, const ObjMaterials *om = nullptr);
// cache key of (k0, k1, rho, s1, om); materials that are all equal reduce to
// the uniform key
NearKey near_key(const bem_mesh *m, double2 k0, double2 k1, double rho, int s1,
                 const ObjMaterials *om);
// hmat.hip: hierarchical (ACA) form of the far part of B
struct HMatStats {
    int n_clusters = 0, n_admissible = 0, n_dense = 0, max_rank = 0;
    int split_blocks = 0;   // admissible blocks split after kmax terms
    double mean_rank = 0, admissible_fraction = 0, eta = 0, tol = 0, setup_seconds = 0;
    double alpha = 1;       // scaling of the phi rows and columns in the cross approximation
    int leaf = 0, kmax = 0;
    int64_t bytes = 0, lowrank_bytes = 0, dense_bytes = 0;
};
std::unique_ptr<HMatrix, HMatDeleter> hmat_build(bem_mesh *m, const NearOperator &nf, double2 k0,
                                                 hipStream_t s);
void hmat_apply(HMatrix &H, bem_mesh *m, const NearOperator &nf, const double2 *x, double2 *y,
                hipStream_t s);
int64_t hmat_bytes(const HMatrix &h);
const HMatStats &hmat_stats(const HMatrix &h);
// cached per wavenumber pair and materials (built on first use)
// device bytes of the compressed operator: those of the cached one, else an
// upper estimate (a quarter of the complex64 dense operator, at least 1 GiB)
int64_t hmat_bytes_estimate(const bem_mesh *m, double2 k0, double2 k1, double rho);
HMatrix &hmat_get(bem_mesh *m, double2 k0, double2 k1, double rho, hipStream_t s, int s1 = 1,
                  const ObjMaterials *om = nullptr);
// dense.hip
int64_t dense_bytes(const bem_mesh *m, bool fp64 = false);
int64_t dense_assembly_scratch_bytes(const bem_mesh *m, bool fp64 = false);
// operator and assembly scratch of a mesh of N vertices and T triangles
int64_t dense_need_bytes(int64_t N, int64_t T, bool fp64);
// The assembled operator of m from its DenseShare (assembled once by the
// first replica that needs it; held while the returned pointer lives).
std::shared_ptr<const DenseOperator> dense_share_get(bem_mesh *m, double2 k0, double2 k1,
                                                     double rho, hipStream_t s, int s1,
                                                     const ObjMaterials *om, int kind);
// complex64 operator rounded from the complex128 one (both cached on m)
const DenseOperator &dense_get_rounded(bem_mesh *m, double2 k0, double2 k1, double rho,
                                       hipStream_t s, int s1, const ObjMaterials *om);
std::unique_ptr<DenseOperator> dense_assemble(bem_mesh *m, const NearOperator &nf, double2 k0,
                                              double2 k1, double rho, hipStream_t s,
                                              bool fp64 = false);
// fp64: the complex128 operator (FP64 assembly, kept apart from the
// complex64 one)
const DenseOperator &dense_get(bem_mesh *m, double2 k0, double2 k1, double rho, hipStream_t s,
                               int s1 = 1, const ObjMaterials *om = nullptr, bool fp64 = false);
// y_r = B x_r, r < R (x, y RHS-major [R][2N]): multi-vector product reading B
// once per 8 right-hand sides
void dense_gemv(const DenseOperator &op, const double2 *x, double2 *y, int R, DevBuf<float2> &xs,
                hipStream_t s, bool skinny = true);
// Y = B X for R right-hand sides (x, y RHS-major [R][2N]) on MFMA
void dense_gemm(const DenseOperator &op, const double2 *x, double2 *y, int R, hipStream_t s);
int64_t dense_gemm_scratch_bytes(const bem_mesh *m, int R);
// MFMA product from tuning().dense_gemm_min_rhs right-hand sides, else dense_gemv
void dense_apply(const DenseOperator &op, const double2 *x, double2 *y, int R,
                 DevBuf<float2> &xs, hipStream_t s, const TuneEntry *forced = nullptr);

// Issue rates (lane operations per second over the device) of v_fma_f32,
// v_sin_f32, v_cos_f32, v_rsq_f32 and v_fma_f64; rates[5].
void valu_rates(double *rates, hipStream_t s);

// field.hip: total field at n points (device [n][3]) for the solution x of
// the plane wave along dir (host [3]); out device [n]; region device [n] or
// NULL (0 outside, m + 1 inside object m)
void field_eval(bem_mesh *m, double2 k0, double2 k1, double rho, const double *dir,
                const double2 *x, const double *pts, int64_t n, double2 *out, int32_t *region,
                hipStream_t s, const ObjMaterials *om = nullptr);

// mesh.cpp
void mesh_build(bem_mesh *m, const double *P, int64_t N, const int32_t *tri,
                int64_t T, const int32_t *obj);
// rhs.hip
void rhs_project(bem_mesh *m, double2 k0, const double *dirs, int n, double2 *f,
                 hipStream_t s);
void far_field_eval(bem_mesh *m, double2 k0, const double2 *x, const double *dirs,
                    int n, double2 *out, hipStream_t s);
// osrc.cpp / osrc.hip
// k_obj: wavenumber of each object when they differ (nullptr: k for all)
OsrcState &osrc_get(bem_mesh *m, int np, double theta, double2 k,
                    const std::vector<double2> &keps_obj, hipStream_t s,
                    const std::vector<double2> *k_obj = nullptr);
// the cached state of these parameters, or nullptr (nothing is created)
OsrcState *osrc_find(bem_mesh *m, int np, double theta, double2 k,
                     const std::vector<double2> &keps_obj);
// Work memory of an apply of R right-hand sides: work [R][np + 2][n],
// obuf [R][np + 3][n], wbuf [R][2][n] (complex128 each).  nullptr: the
// state's own buffers, grown to R on demand.
struct OsrcScratch {
    double2 *work, *obuf, *wbuf;
};
// complex128 entries of OsrcScratch per right-hand side (the mesh's OSRC
// symbolic state must exist)
int64_t osrc_scratch_per_rhs(const bem_mesh *m, int np);
// work entries of one system of the solves (n + partial sums); state must exist
int64_t osrc_work_len(const bem_mesh *m);
// the scratch of `batch` right-hand sides laid out from base
OsrcScratch osrc_scratch_at(const bem_mesh *m, int np, int batch, double2 *base);
// R right-hand sides, [R][2N] contiguous each
void osrc_apply_strong(bem_mesh *m, OsrcState &st, const double2 *x, double2 *y, int R,
                       hipStream_t s, const OsrcScratch *scr = nullptr);
void osrc_apply_from_weak(bem_mesh *m, OsrcState &st, const double2 *yw, double2 *z, int R,
                          hipStream_t s, const OsrcScratch *scr = nullptr);
void osrc_mass_solve(bem_mesh *m, OsrcState &st, const double2 *x, double2 *y,
                     int nblocks, hipStream_t s);
// symbolic analysis of the OSRC systems (once per mesh handle)
void osrc_prepare(bem_mesh *m);
// device bytes of one OSRC factor state with np Pade terms, sized for R
// right-hand sides per apply (runs the symbolic analysis if needed)
int64_t osrc_state_bytes(bem_mesh *m, int np, int R);
// solve.cpp
// Validated OSRC-preconditioned solve (the body of pmchwt_solve); throws Error.
// om: per-object interior materials (nullptr: k1, rho for every object)
int solve_run(bem_mesh *m, double2 k0, double2 k1, double rho, const double *dirs,
              int n_waves, double tol, const bem_solve_opts &o, double2 *solution,
              bem_solve_info *info, hipStream_t s, const ObjMaterials *om = nullptr);
// one valid (k_m, rho_m) per object, else throws BEM_E_INVAL
void check_materials(const bem_mesh *m, const ObjMaterials &om);
void solve_check(const bem_mesh *m, double2 k0, double2 k1, double rho, const double *dirs,
                 int n_waves, double tol, const bem_solve_opts &o);
// Upper bound of the device memory one solve adds to a mesh handle with no
// cached state (near field, OSRC factors, scratch, the dense operator when
// o.path == 1 and FP32, the Krylov basis for o.maxiter iterations).
int64_t solve_footprint(bem_mesh *m, double2 k0, double2 k1, double rho,
                        const bem_solve_opts &o, int n_waves);
// mesh.cpp: release cached operators and scratch (geometry and the OSRC
// symbolic analysis stay)
void mesh_trim(bem_mesh *m);
// build m->parts / m->part_vidx if not yet built (several objects)
void mesh_parts(bem_mesh *m);
// profiling (api.cpp)
// Device memory a solve takes beyond its admission footprint (its Krylov
// basis as it grows) is reported, while a ReserveScope is alive on the
// thread, to its hook: the serving loop accounts it against its budget.
using ReserveHook = void (*)(void *ctx, int64_t delta_bytes);
struct ReserveScope {
    ReserveScope(ReserveHook hook, void *ctx);
    ~ReserveScope();
    ReserveHook prev_hook;
    void *prev_ctx;
};
void reserve_bytes(int64_t delta_bytes);

// While one is alive on a thread, Timer records nothing (no HIP events are
// created): for calls that must not allocate.
struct NoTimerScope {
    NoTimerScope();
    ~NoTimerScope();
    bool prev;
};

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    const char *name = nullptr;
    hipStream_t s = nullptr;
    Timer(const char *kernel, hipStream_t stream);
    ~Timer();
};

}   // namespace bem

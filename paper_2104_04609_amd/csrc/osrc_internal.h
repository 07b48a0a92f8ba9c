// Internal types of the OSRC preconditioner (host + device launch interface).
#pragma once

#include "bem_internal.h"
#include "sparse_ldl.h"

namespace bem {

constexpr int PADE_MAX = 32;

struct PadeCoef {
    int np;
    double2 C0;
    double2 A[PADE_MAX];
};

// Bottom-subtree plan of a batch: subtrees of up to OSRC_SUB_ROWS rows, or
// larger ones when they still give OSRC_SUB_MIN_GROUPS workgroups (subtrees
// x systems x vectors).
constexpr int OSRC_SUB_ROWS = 2048;
constexpr int OSRC_SUB_MIN_GROUPS = 1024;

// Largest dissection block (rows) a level workgroup can hold in LDS.
constexpr int LDL_MAX_BLOCK = 4096;

// Everything a solve kernel needs about one row, in one 48-byte record (one
// round trip instead of a chain of dependent index loads).
struct alignas(16) LdlRow {
    int j, perm, s0, w;    // row (new order), perm[j], first row and width of its block
    int fx, fy, bx, by;    // forward CSR / backward CSC external entry ranges
    int doff, rr, bsplit, pad;   // dense inverse offset of the block, row within the
                                 // block, first CSC position in the top (two-part solve)
};

// Deepest subtree (heights) of the two-part solve.
constexpr int LDL_SPLIT_MAX_H = 48;

// Device view of the shared LDL^T structure plus the numeric factors.
struct LdlDev {
    int n;
    int64_t nnz;              // strict lower entries of L
    int64_t ndense;           // entries of the dense block inverses
    const int32_t *perm;      // perm[new] = old
    const int32_t *Rj;        // CSR column indices of L (forward sweep)
    const int32_t *Li;        // CSC row indices of L (backward sweep with L^T)
    int nlev;                 // levels of the dissection tree
    const int32_t *lbcount;   // host: blocks per level
    const int32_t *lrcount;   // host: rows per level
    const double2 *Dinv;      // [factors][n]
    const double2 *Lcsr;      // [factors][nnz]
    const double2 *Lcsc;      // [factors][nnz]
    const double2 *invL;      // [factors][ndense]
    const double2 *invLT;     // [factors][ndense]
    int64_t wlen;             // work length per system: n + partial sums of the split solve
    const LdlRow *jrow;       // row descriptors by row j
    const LdlRow *lrowd;      // row descriptors in level order (rows of the blocks of height l)
    const int4 *lblkd;        // blocks in level order: {s0, w, doff, 0}
    const int32_t *lptr_h;    // host: level l's rows lrowd[lptr_h[l] .. lptr_h[l+1])
    const int32_t *lbptr_h;   // host: level l's blocks lblkd[lbptr_h[l] .. lbptr_h[l+1])
    const int64_t *lext_f;    // host: external entries of each level, forward / backward
    const int64_t *lext_b;
};

// Levels whose rows average more external entries than this run their
// external updates with one workgroup per row.
constexpr int LDL_WIDE_EXT = 128;

// Device view of the two-part schedule (LdlSplit): bottom subtrees solved
// in LDS by one workgroup each, the top part by one workgroup (top_single)
// or level by level.
struct LdlSplitDev {
    int ok;                   // 0: level-by-level solve only
    int H, nsub, ntop, nht;   // cut height, subtrees, top rows, top heights
    int top_single;           // 1: the top part in one workgroup
    int top_levels;           // 1: the top part by the level kernels of the one-launch-
                              // per-level schedule (no partial sums)
    int sub_rows;             // largest subtree (rows)
    int hrows;                // most rows of one (subtree or top part, height)
    int desc_lds;             // 1: the subtree kernels keep their rows' descriptors in LDS
    const int32_t *sub_r0, *sub_r1, *sub_hptr, *srow;
    const LdlRow *sdesc;      // row descriptors in srow order (bsplit filled)
    const int32_t *top_row, *top_hptr, *tlist;
    const int32_t *part_b, *part_e;
    const int32_t *tf_ptr, *tf_pos, *tf_col, *tb_ptr, *tb_pos, *tb_row;
    const int32_t *bsplit;
};

// One system solve: out = scale * A_factor^{-1} in (vectors of length n).
struct SolveTask {
    int factor;
    const double2 *in;
    double2 *out;
    double2 scale;
    double2 *work;
};

// One two-part schedule and its device copies.
struct SplitSchedule {
    LdlSplit plan;
    DevBuf<int32_t> sub_r0, sub_r1, sub_hptr, srow, top_row, top_hptr, tlist, part_b, part_e,
        tf_ptr, tf_pos, tf_col, tb_ptr, tb_pos, tb_row, bsplit;
    DevBuf<LdlRow> sdesc;
    int top_single = 0;
    int top_levels = 0;   // the top part by the level kernels (no partial sums)
    int rows = 0;         // subtree rows the plan was made for
    int hrows = 0;   // most rows of one (subtree or top part, height)
    int desc_lds = 0;   // row descriptors of a subtree fit in LDS
    int64_t bytes() const;
};

// Mesh-level (parameter-independent) OSRC data: P1 vertex graph, mass and
// stiffness values, ordering and symbolic LDL^T, and their device copies.
struct OsrcSymbolicState {
    int n = 0;
    std::vector<int32_t> gptr, gcol;
    std::vector<double> Mv, Sv;
    LdlSymbolic sym;
    DevBuf<int32_t> gptr_d, gcol_d, perm_d, Rj_d, Li_d;
    std::vector<int32_t> lbcount, lrcount;   // blocks and rows per level (host)
    std::vector<int32_t> lptr_h, lbptr_h;
    std::vector<int64_t> lext_f, lext_b;
    DevBuf<LdlRow> jrow_d, lrowd_d;
    DevBuf<int4> lblkd_d;
    // two-part schedules of the block solves: `split` with partial sums of the
    // top rows (osrc.split 2), `bottom` with the top part by the level kernels
    // (nbottom plans of growing subtrees, osrc.split 1 and 3)
    int split_mode = 1;
    SplitSchedule split;
    SplitSchedule bottom[4];
    int nbottom = 0;
    int64_t wlen = 0;   // work length per system (n + partial sums)
    DevBuf<double> Mv_d, Sv_d;
    int64_t bytes() const;
};

struct OsrcState {
    int np = 0;
    int64_t wlen = 0;            // work length per system (OsrcSymbolicState::wlen)
    double2 k{0, 0};
    PadeCoef pc{};               // C_0, A_j of the Pade approximant
    PadeCoef pf{};               // partial fractions: C_0', A_j / B_j
    PadeCoef qf{};               // R(X)(I + X)^{-1} over (I + X)^{-1} and the shifts
    std::vector<double2> B;      // Pade B_j
    int nfactors = 0;            // np shifts, (M - S/k_eps^2), M
    DevBuf<double2> cvert;       // 1/k_eps^2 of each vertex's object
    DevBuf<double2> ikv, iikv;   // ik and 1/(ik) per vertex (objects with their own k), else empty
    DevBuf<double2> Dinv, Lcsr, Lcsc, invL, invLT;
    // per right-hand side r of a batched apply (capacity `batch`):
    DevBuf<double2> work;        // [r][np + 2][n] solve work vectors
    DevBuf<double2> obuf;        // [r][np + 3][n]: s_0..s_{np-1}, u, v, M v
    DevBuf<double2> wbuf;        // [r][2][n] weak vectors (strong-form entry)
    int batch = 0;
    void ensure_batch(int R);
    int64_t bytes() const;
};

// Task list passed by value as a kernel argument (at most PADE_MAX + 2
// systems per right-hand side).  A launch runs nbase x R tasks: task
// (r, b) is t[b] with in/out/work advanced by r times the strides.
struct TaskList {
    SolveTask t[PADE_MAX + 2];
    int nbase;
    int64_t in_stride, out_stride, work_stride;
};

void launch_ldl_solve(const LdlDev &L, const LdlSplitDev &P, TaskList tasks, int ntasks,
                      int nrhs, hipStream_t s);
// rows of LDS a bottom-subtree workgroup may hold on this device
int ldl_split_max_sub_rows();
// LDS of a split workgroup: `rows` rows, `hrows` staged dense results and
// their indices, `desc_rows` row descriptors; the device's limit
size_t ldl_split_lds(int rows, int hrows, int desc_rows);
int ldl_split_max_lds();
// offset (in double2 past the staged results) of the descriptors, 16-byte aligned
__host__ __device__ inline int ldl_split_desc_off(int hrows) { return hrows + (hrows * 4 + 15) / 16; }
// out_r = alpha (C0 u_r - sum_j A_j s_{r,j})   (elementwise, r < nrhs):
// u_r = u + r ustride, s_{r,j} = sv + r vstride + j sstride, out_r = out + r ostride
void launch_pade_sum(int n, const PadeCoef &pc, double2 alpha, const double2 *alpha_v,
                     const double2 *u, int64_t ustride, const double2 *sv, int64_t sstride,
                     int64_t vstride, double2 *out, int64_t ostride, int nrhs, hipStream_t s);
// both in one launch: npade Pade sums and nspmv mass products
// (mout_b = M in_b, in_b = in + b istride, mout_b = mout + b mstride)
void launch_pade_sum_spmv(int n, const PadeCoef &pc, double2 alpha, const double2 *alpha_v,
                          const double2 *u, int64_t ustride, const double2 *sv, int64_t sstride,
                          int64_t vstride, double2 *out, int64_t ostride, int npade,
                          const int32_t *gptr, const int32_t *gcol, const double *V,
                          const double2 *in, int64_t istride, double2 *mout, int64_t mstride,
                          int nspmv, hipStream_t s);
// two Pade sums per right-hand side in one launch: out_r = alpha (C0 u_r -
// sum_j A_j s_{r,j}) by pc (s_{r,j} = sv + r ostride + j sstride) and out2_r
// likewise by pc2 from u2, sv2 (same strides)
void launch_pade_pair(int n, const PadeCoef &pc, double2 alpha, const double2 *alpha_v,
                      const double2 *u, int64_t ustride, const double2 *sv, int64_t sstride,
                      int64_t vstride, double2 *out, int64_t ostride, const PadeCoef &pc2,
                      double2 alpha2, const double2 *alpha2_v, const double2 *u2,
                      const double2 *sv2, double2 *out2, int nrhs, hipStream_t s);
// out_b = V in_b for b < nblk, in_b = in + b istride, out_b = out + b ostride
void launch_spmv_real(int n, int nblk, const int32_t *gptr, const int32_t *gcol,
                      const double *V, const double2 *in, int64_t istride, double2 *out,
                      int64_t ostride, hipStream_t s);

}   // namespace bem

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

// Device view of the shared LDL^T structure plus the numeric factors.
struct LdlDev {
    int n;
    int64_t nnz;            // strict lower entries of L
    const int32_t *perm;    // perm[new] = old
    const int32_t *Rp, *Rj; // CSR of L (forward sweep)
    const int32_t *Lp, *Li; // CSC of L (backward sweep with L^T)
    const int32_t *fptr, *frow, *bptr, *brow;
    int nfl, nbl;
    const double2 *Dinv;    // [factors][n]
    const double2 *Lcsr;    // [factors][nnz]
    const double2 *Lcsc;    // [factors][nnz]
};

// One system solve: out = scale * A_factor^{-1} in (vectors of length n).
struct SolveTask {
    int factor;
    const double2 *in;
    double2 *out;
    double2 scale;
    double2 *work;
};

// Mesh-level (parameter-independent) OSRC data: P1 vertex graph, mass and
// stiffness values, ordering and symbolic LDL^T, and their device copies.
struct OsrcSymbolicState {
    int n = 0;
    std::vector<int32_t> gptr, gcol;
    std::vector<double> Mv, Sv;
    LdlSymbolic sym;
    DevBuf<int32_t> gptr_d, gcol_d, perm_d, Rp_d, Rj_d, Lp_d, Li_d, fptr_d, frow_d, bptr_d,
        brow_d;
    DevBuf<double> Mv_d, Sv_d;
    int64_t bytes() const;
};

struct OsrcState {
    int np = 0;
    double2 k{0, 0};
    PadeCoef pc{};
    std::vector<double2> B;      // Pade B_j
    int nfactors = 0;            // np shifts, (M - S/k_eps^2), M
    DevBuf<double2> cvert;       // 1/k_eps^2 of each vertex's object
    DevBuf<double2> Dinv, Lcsr, Lcsc;
    DevBuf<double2> work;        // (np + 1) x n solve work vectors
    DevBuf<double2> sbuf;        // np x n shifted-solve outputs
    DevBuf<double2> tmp;         // 4 x n
    DevBuf<double2> wbuf;        // 2 x n weak vectors (strong-form entry)
    int64_t bytes() const;
};

// Task list passed by value as a kernel argument (at most PADE_MAX + 1 systems).
struct TaskList {
    SolveTask t[PADE_MAX + 1];
};

void launch_ldl_solve(const LdlDev &L, const TaskList &tasks, int ntasks, hipStream_t s);
void launch_pade_combine(int n, const int32_t *gptr, const int32_t *gcol, const double *Sv,
                         const double2 *cvert, const PadeCoef &pc, const double2 *in,
                         const double2 *sv, int64_t sstride, double2 *out, hipStream_t s);
void launch_spmv_real(int n, int nblk, const int32_t *gptr, const int32_t *gcol,
                      const double *V, const double2 *in, double2 *out, hipStream_t s);

}   // namespace bem

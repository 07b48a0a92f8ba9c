// Sparse complex-symmetric LDL^T (no pivoting) sharing one symbolic
// structure across many numeric factorisations, as needed by the OSRC Pade
// systems (M - beta_j S), which all have the P1 vertex-graph pattern (the
// paper computes one sparse factorisation per system once, Sec. 2.6).
//
// Host-only C++ (no HIP): ordering, symbolic analysis, numeric factorisation
// and a reference triangular solve.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace bem {

using cd = std::complex<double>;

struct LdlSymbolic {
    int n = 0;
    std::vector<int32_t> perm;    // perm[new] = old
    std::vector<int32_t> iperm;   // iperm[old] = new
    // permuted lower triangle of A (incl. diagonal), CSC: column j holds rows >= j
    std::vector<int32_t> Ap, Ai, Asrc;   // Asrc: position in the caller's CSR values
    // strict lower triangle of L, CSC (column j: rows > j, ascending)
    std::vector<int32_t> Lp, Li;
    // the same entries by rows (CSR: row i: columns < i, ascending) and the CSC
    // position of each CSR entry
    std::vector<int32_t> Rp, Rj, Rmap;
    std::vector<int32_t> parent;  // elimination tree
    // level schedules: forward (by height in the tree, leaves first) and
    // backward (by depth, roots first)
    std::vector<int32_t> fptr, frow, bptr, brow;
    int64_t nnzL() const { return Lp.empty() ? 0 : Lp.back(); }
};

// Geometric nested dissection of an undirected graph (CSR incl. diagonal)
// with vertex coordinates xyz[3n]; vertices are split at the median of the
// widest coordinate, the separator is the set of vertices on one side with a
// neighbour on the other, ordered last.  `group` (size n) keeps groups
// (objects) apart: each group is dissected on its own.
std::vector<int32_t> nested_dissection(int n, const std::vector<int32_t> &ptr,
                                       const std::vector<int32_t> &col,
                                       const std::vector<double> &xyz,
                                       const std::vector<int32_t> &group, int leaf = 48);

// Symbolic analysis of a symmetric pattern (CSR incl. diagonal, both
// triangles) under the permutation perm.
LdlSymbolic ldl_symbolic(int n, const std::vector<int32_t> &ptr,
                         const std::vector<int32_t> &col, const std::vector<int32_t> &perm);

// Numeric factorisation: vals are the caller's CSR values (same pattern as
// given to ldl_symbolic).  Outputs D[n] and the strict lower L values in CSC
// order (Lx[nnzL]).  Returns false on a zero pivot.
bool ldl_numeric(const LdlSymbolic &S, const std::vector<cd> &vals, std::vector<cd> &D,
                 std::vector<cd> &Lx);

// Reference solve A x = b in the original ordering (tests and debugging).
void ldl_solve_host(const LdlSymbolic &S, const std::vector<cd> &D, const std::vector<cd> &Lx,
                    const std::vector<cd> &b, std::vector<cd> &x);

}   // namespace bem

// Sparse complex-symmetric LDL^T (no pivoting) sharing one symbolic
// structure across many numeric factorisations, as needed by the OSRC Pade
// systems (M - beta_j S), which all have the P1 vertex-graph pattern (the
// paper computes one sparse factorisation per system once, Sec. 2.7).
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
    // Dissection blocks (leaves and separators) in the new ordering: block b
    // holds rows [bstart[b], bstart[b+1]); its height in the dissection tree
    // (leaves 0) makes the level schedule of the block solves.  Rows of one
    // block only reference rows of the same block or of its descendants.
    std::vector<int32_t> bstart, bheight, blk;   // blk[row] = block id
    std::vector<int64_t> doff;                   // dense offset of block b (sum of w^2)
    int64_t ndense = 0;
    // level schedule: rows of all blocks of height l are lrow[lptr[l] .. lptr[l+1])
    std::vector<int32_t> lptr, lrow;
    // external parts of L: forward row j uses CSR entries [Rp[j], fext[j]) (columns
    // before its block); backward column j uses CSC entries [bext[j], Lp[j+1])
    // (rows after its block)
    std::vector<int32_t> fext, bext;
    bool blocks_ok = true;   // every external entry points to a lower level
    int64_t nnzL() const { return Lp.empty() ? 0 : Lp.back(); }
};

struct NdOrder {
    std::vector<int32_t> order;    // order[new] = old
    std::vector<int32_t> bstart;   // block boundaries (size nblocks + 1)
    std::vector<int32_t> bheight;  // block heights in the dissection tree
};

// Geometric nested dissection of an undirected graph (CSR incl. diagonal)
// with vertex coordinates xyz[3n]; vertices are split at the median of the
// widest coordinate, the separator is the set of vertices on one side with a
// neighbour on the other, ordered last.  `group` (size n) keeps groups
// (objects) apart: each group is dissected on its own.
// Leaves (at most `leaf` vertices) and separators are the blocks.
NdOrder nested_dissection(int n, const std::vector<int32_t> &ptr, const std::vector<int32_t> &col,
                          const std::vector<double> &xyz, const std::vector<int32_t> &group,
                          int leaf = 48);

// Symbolic analysis of a symmetric pattern (CSR incl. diagonal, both
// triangles) under the dissection ordering nd.
LdlSymbolic ldl_symbolic(int n, const std::vector<int32_t> &ptr,
                         const std::vector<int32_t> &col, const NdOrder &nd);

// Numeric factorisation: vals are the caller's CSR values (same pattern as
// given to ldl_symbolic).  Outputs D[n] and the strict lower L values in CSC
// order (Lx[nnzL]).  Returns false on a zero pivot.
bool ldl_numeric(const LdlSymbolic &S, const std::vector<cd> &vals, std::vector<cd> &D,
                 std::vector<cd> &Lx);

// Inverses of the unit lower-triangular diagonal blocks L_BB of every
// dissection block, dense row-major w x w at doff[b]: invL and its transpose.
void ldl_block_inverses(const LdlSymbolic &S, const std::vector<cd> &Lx, std::vector<cd> &invL,
                        std::vector<cd> &invLT);

// Block solve in the original ordering, the algorithm the device runs:
// per level, y_B -= L_B,ext y_ext then y_B = inv(L_BB) y_B (forward), D^{-1},
// then the transposed sweep from the top level down.
void ldl_solve_blocks_host(const LdlSymbolic &S, const std::vector<cd> &D,
                           const std::vector<cd> &Lx, const std::vector<cd> &invL,
                           const std::vector<cd> &invLT, const std::vector<cd> &b,
                           std::vector<cd> &x);

// Reference solve A x = b in the original ordering (tests and debugging).
void ldl_solve_host(const LdlSymbolic &S, const std::vector<cd> &D, const std::vector<cd> &Lx,
                    const std::vector<cd> &b, std::vector<cd> &x);

}   // namespace bem

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
    // the subtree rooted at block b is the contiguous block range
    // [bfirst[b], b] (rows [bstart[bfirst[b]], bstart[b + 1]))
    std::vector<int32_t> bfirst;
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
    std::vector<int32_t> bfirst;   // first block of the subtree rooted at each block
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

// Two-part schedule of the block solves.  The dissection tree is cut at
// height H: the maximal subtrees of blocks of height < H ("bottom"; rows
// [r0, r1) each, contiguous) are solved independently, each by one device
// workgroup holding its rows in LDS; the blocks of height >= H ("top") are
// solved by one workgroup per system.  A top row's forward external update
// is split into its entries in each subtree (partial sums formed by the
// subtree's workgroup) and its entries inside the top part.  H is the
// largest height at which every subtree has at most sub_max_rows rows, the
// top part at most top_max_rows rows and every (subtree or top, height)
// group at most phase_max_rows rows; ok = false if there is none.
struct LdlSplit {
    bool ok = false;
    int H = 0, hmax = 0, nsub = 0, ntop = 0;
    int max_sub_rows = 0;
    std::vector<int32_t> sub_r0, sub_r1;   // subtree s: rows [r0, r1)
    std::vector<int32_t> sub_hptr;         // [nsub][H + 1]: subtree s, height h -> srow range
    std::vector<int32_t> srow;             // bottom rows by (subtree, height), ascending
    std::vector<int32_t> top_row;          // top rows ascending (global); t = local index
    std::vector<int32_t> top_hptr;         // [hmax - H + 2]: height H + i -> tlist range
    std::vector<int32_t> tlist;            // top local indices by height, ascending
    std::vector<int32_t> part_b, part_e;   // [nsub][ntop]: CSR entries of top row t in subtree s
    std::vector<int32_t> tf_ptr, tf_pos, tf_col;   // top row t: forward entries in the top
                                                   // part (CSR position, local column)
    std::vector<int32_t> tb_ptr, tb_pos, tb_row;   // top row t: backward entries (CSC
                                                   // position, local row); all in the top
    std::vector<int32_t> bsplit;           // bottom row j: first CSC position in
                                           // [bext[j], Lp[j+1]) whose row is in the top
};
LdlSplit ldl_split_plan(const LdlSymbolic &S, int sub_max_rows, int top_max_rows,
                        int phase_max_rows);

// The two-part block solve on the host (the order of the device kernels).
void ldl_solve_split_host(const LdlSymbolic &S, const LdlSplit &P, const std::vector<cd> &D,
                          const std::vector<cd> &Lx, const std::vector<cd> &invL,
                          const std::vector<cd> &invLT, const std::vector<cd> &b,
                          std::vector<cd> &x);

// Reference solve A x = b in the original ordering (tests and debugging).
void ldl_solve_host(const LdlSymbolic &S, const std::vector<cd> &D, const std::vector<cd> &Lx,
                    const std::vector<cd> &b, std::vector<cd> &x);

}   // namespace bem

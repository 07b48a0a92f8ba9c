// Hierarchical (H-matrix) form of the far part of the permuted PMCHWT
// operator, for meshes whose dense operator does not fit and whose
// matrix-free product is too slow (the paper compresses every operator as an
// H-matrix with tolerance 1e-5, Sec. 3.1, to reach its 145 338-node mesh,
// Sec. 3.6).
//
// Vertices are ordered along a binary cluster tree (median bisection of the
// widest bounding-box axis, leaves of at most `leaf` vertices).  A pair of
// clusters is admissible when max(diam) <= eta dist of their bounding boxes,
// each box covering the triangles of the cluster's vertices (so that no
// triangle pair of an admissible block shares a vertex).  On an admissible
// pair the 2m x 2n block of B (rows [psi-row; phi-row] of the m test
// vertices, columns [psi; phi] of the n trial vertices) is approximated by
// adaptive cross approximation with partial pivoting, U V^T with the rank
// chosen so that the last cross ||u_k|| ||v_k|| <= tol ||U V^T||_F; pairs of
// leaves that are not admissible are stored dense.  Entries are the far-field
// entries of the dense assembly (tri_vertex_entries: the 6x6 rule over the
// triangle pairs sharing no vertex, FP32); the triangle pairs sharing a
// vertex stay in the FP64 near-field operator.
//
// Product y = B x: z_b = V_b^T x_sigma per admissible block, then per leaf
// of the test tree (one workgroup, fixed order: the admissible blocks of its
// ancestors from the root down, then its dense blocks) y_rows = sum U_b z_b +
// sum D x, FP64 sums of FP32 entries; finally the near-field CSR.  The result
// is deterministic.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "bem_internal.h"
#include "entries.h"

namespace bem {

namespace {

using namespace entries;

constexpr int ACA_THREADS = 256;
constexpr int ROW_THREADS = 128;   // product: one thread per row of a leaf (2 x leaf <= 128)

// ---------------------------------------------------------------- host tree
struct Cluster {
    int v0 = 0, v1 = 0;        // tree positions [v0, v1)
    int child[2] = {-1, -1};
    int parent = -1;
    double lo[3], hi[3];       // box of the triangles of its vertices
};

double box_diam(const Cluster &c) {
    double s = 0;
    for (int a = 0; a < 3; a++) s += (c.hi[a] - c.lo[a]) * (c.hi[a] - c.lo[a]);
    return std::sqrt(s);
}
double box_dist(const Cluster &a, const Cluster &b) {
    double s = 0;
    for (int k = 0; k < 3; k++) {
        const double d = std::max(0.0, std::max(a.lo[k] - b.hi[k], b.lo[k] - a.hi[k]));
        s += d * d;
    }
    return std::sqrt(s);
}

struct TreeBuilder {
    const bem_mesh *m;
    int leaf;
    std::vector<int32_t> order;   // tree position -> vertex
    std::vector<Cluster> cl;
    std::vector<double> tlo, thi;   // per vertex: box of its star
    int build(int v0, int v1, int parent) {
        Cluster c;
        c.v0 = v0;
        c.v1 = v1;
        c.parent = parent;
        for (int a = 0; a < 3; a++) {
            c.lo[a] = 1e300;
            c.hi[a] = -1e300;
        }
        for (int p = v0; p < v1; p++)
            for (int a = 0; a < 3; a++) {
                c.lo[a] = std::min(c.lo[a], tlo[3 * order[p] + a]);
                c.hi[a] = std::max(c.hi[a], thi[3 * order[p] + a]);
            }
        const int id = (int)cl.size();
        cl.push_back(c);
        if (v1 - v0 > leaf) {
            // split the vertices at the median of the widest axis of their positions
            double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
            for (int p = v0; p < v1; p++)
                for (int a = 0; a < 3; a++) {
                    lo[a] = std::min(lo[a], m->P[3 * order[p] + a]);
                    hi[a] = std::max(hi[a], m->P[3 * order[p] + a]);
                }
            int ax = 0;
            for (int a = 1; a < 3; a++)
                if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
            const int mid = (v0 + v1) / 2;
            std::nth_element(order.begin() + v0, order.begin() + mid, order.begin() + v1,
                             [&](int a, int b) {
                                 const double xa = m->P[3 * a + ax], xb = m->P[3 * b + ax];
                                 return xa < xb || (xa == xb && a < b);
                             });
            const int c0 = build(v0, mid, id);
            const int c1 = build(mid, v1, id);
            cl[id].child[0] = c0;
            cl[id].child[1] = c1;
        }
        return id;
    }
};

struct BlockLists {
    std::vector<std::pair<int, int>> adm, nearb;   // (row cluster, col cluster)
};

void build_blocks(const std::vector<Cluster> &cl, int a, int b, double eta, BlockLists &out) {
    const Cluster &A = cl[a], &B = cl[b];
    const double dist = box_dist(A, B);
    if (dist > 0 && std::max(box_diam(A), box_diam(B)) <= eta * dist) {
        out.adm.push_back({a, b});
        return;
    }
    const bool la = A.child[0] < 0, lb = B.child[0] < 0;
    if (la && lb) {
        out.nearb.push_back({a, b});
        return;
    }
    if (la) {
        for (int c : B.child) build_blocks(cl, a, c, eta, out);
    } else if (lb) {
        for (int c : A.child) build_blocks(cl, c, b, eta, out);
    } else {
        for (int c : A.child)
            for (int d : B.child) build_blocks(cl, c, d, eta, out);
    }
}

// ---------------------------------------------------------------- device
struct EntryArgs {
    const double *geo;     // FP64 geometry: entries are evaluated in FP64
    const double *tst;
    const int32_t *tobj, *tri, *star_ptr, *star_idx;
    const int32_t *perm;   // tree position -> vertex
    DCoefT<double> cf;
    const DIntT<double> *itab;
    // per cluster c: its triangles (those with a vertex in it) at
    // ct_idx[ct_ptr[c] .. ct_ptr[c + 1]), and for its p-th vertex the slots
    // (place in that list * 3 + local index) at
    // cv_slot[cv_ptr[cv_off[c] + p] .. cv_ptr[cv_off[c] + p + 1])
    const int32_t *ct_ptr, *ct_idx;
    const int64_t *cv_off;
    const int32_t *cv_ptr, *cv_slot;
};

// The four blocks of B_far(i, j) (test vertex i, trial vertex j, original
// ids): out[blk] for blk = 2 c + d (c: psi-/phi-row, d: psi/phi column).
template <bool CK0, bool CK1, bool MULTI>
__device__ void vertex_entries(const EntryArgs &A, int i, int j, const double2 *etab,
                               float2 out[4]) {
    double accr[4] = {0, 0, 0, 0}, acci[4] = {0, 0, 0, 0};
    for (int e = A.star_ptr[i]; e < A.star_ptr[i + 1]; e++) {
        const int ta = A.star_idx[e];
        const int t = ta / 3, a = ta - 3 * t;
        double px[6], py[6], pz[6], ntx, nty, ntz, ct, cu[9];
        load_test(A.geo, A.tst, t, px, py, pz, ntx, nty, ntz, ct, cu);
        double outr[12], outi[12];
        tri_vertex_entries<double, CK0, CK1, MULTI, false>(A.geo, A.tst, A.tobj, A.tri,
                                                           A.star_ptr, A.star_idx, t, j, px, py,
                                                           pz, ntx, nty, ntz, ct, cu, A.cf,
                                                           A.itab, etab, outr, outi);
        for (int blk = 0; blk < 4; blk++) {
            accr[blk] += outr[3 * blk + a];
            acci[blk] += outi[3 * blk + a];
        }
    }
    for (int blk = 0; blk < 4; blk++) out[blk] = make_float2((float)accr[blk], (float)acci[blk]);
}

__device__ inline float2 cmulf(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// The four blocks of B_far(i, j) for every vertex i of cluster c (tree
// positions [v0, v0 + m)) against trial vertex j (original id), in two
// workgroup passes: each triangle of the cluster once as test triangle
// (tri_vertex_entries, 12 values into q), then per vertex the sum over its
// triangles in a fixed order.  out(p, blk) receives block blk of vertex p.
template <bool CK0, bool CK1, bool MULTI, class Out>
__device__ void cluster_column(const EntryArgs &A, int c, int m, int j, double2 *q,
                               const double2 *etab, Out out) {
    const int t0 = A.ct_ptr[c], nt = A.ct_ptr[c + 1] - t0;
    for (int k = threadIdx.x; k < nt; k += ACA_THREADS) {
        const int t = A.ct_idx[t0 + k];
        double px[6], py[6], pz[6], ntx, nty, ntz, ct, cu[9];
        load_test(A.geo, A.tst, t, px, py, pz, ntx, nty, ntz, ct, cu);
        double outr[12], outi[12];
        tri_vertex_entries<double, CK0, CK1, MULTI, false>(A.geo, A.tst, A.tobj, A.tri,
                                                           A.star_ptr, A.star_idx, t, j, px, py,
                                                           pz, ntx, nty, ntz, ct, cu, A.cf,
                                                           A.itab, etab, outr, outi);
        for (int e = 0; e < 12; e++) q[(int64_t)12 * k + e] = make_double2(outr[e], outi[e]);
    }
    __syncthreads();
    const int32_t *vp = A.cv_ptr + A.cv_off[c];
    for (int p = threadIdx.x; p < m; p += ACA_THREADS) {
        double accr[4] = {0, 0, 0, 0}, acci[4] = {0, 0, 0, 0};
        for (int e = vp[p]; e < vp[p + 1]; e++) {
            const int sl = A.cv_slot[e];
            const int k = sl / 3, a = sl - 3 * k;
            for (int blk = 0; blk < 4; blk++) {
                const double2 v = q[(int64_t)12 * k + 3 * blk + a];
                accr[blk] += v.x;
                acci[blk] += v.y;
            }
        }
        for (int blk = 0; blk < 4; blk++)
            out(p, blk, make_float2((float)accr[blk], (float)acci[blk]));
    }
    __syncthreads();
}

// Admissible block of the ACA pass.
struct AcaBlock {
    int r0, m, c0, n;    // test cluster [r0, r0 + m), trial cluster [c0, c0 + n) (tree positions)
    int rc, cc;          // the two clusters
    int64_t uoff, voff;  // scratch: U [kmax][2m], V [kmax][2n] (float2)
    int64_t qoff;        // scratch: 12 complex128 values per triangle of the larger cluster list
    int64_t used_off;    // scratch: used-row marks [2m] (int32)
};

// Block-wide reductions (fixed order).
__device__ inline double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = ACA_THREADS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}
// argmax of v over the block (ties: the smaller index; index -1 for v < 0)
__device__ inline void block_argmax(float v, int idx, float *rv, int *ri, float &bv, int &bi) {
    rv[threadIdx.x] = v;
    ri[threadIdx.x] = idx;
    __syncthreads();
    for (int s = ACA_THREADS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const float o = rv[threadIdx.x + s];
            const int oi = ri[threadIdx.x + s];
            if (o > rv[threadIdx.x] || (o == rv[threadIdx.x] && oi >= 0 &&
                                        (ri[threadIdx.x] < 0 || oi < ri[threadIdx.x]))) {
                rv[threadIdx.x] = o;
                ri[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    bv = rv[0];
    bi = ri[0];
    __syncthreads();
}

// Adaptive cross approximation of one admissible block per workgroup.
// rank[b] receives the rank (kmax + 1 if the tolerance was not reached).
template <bool CK0, bool CK1, bool MULTI>
__global__ __launch_bounds__(ACA_THREADS) void aca_kernel(EntryArgs A, const AcaBlock *blocks,
                                                          int kmax, float tol, float alpha,
                                                          float2 *scr, int32_t *used_scr,
                                                          int32_t *rank) {
    __shared__ double red[ACA_THREADS];
    __shared__ float rv[ACA_THREADS];
    __shared__ int ri[ACA_THREADS];
    __shared__ double2 etab[256];
    const AcaBlock B = blocks[blockIdx.x];
    const int m2 = 2 * B.m, n2 = 2 * B.n;
    float2 *U = scr + B.uoff, *V = scr + B.voff;
    double2 *Q = reinterpret_cast<double2 *>(scr + B.qoff);   // qoff even: 16-byte aligned
    int32_t *used = used_scr + B.used_off;
    for (int r = threadIdx.x; r < m2; r += ACA_THREADS) used[r] = 0;
    DM<double>::fill_table(etab);
    __syncthreads();
    double norm2 = 0.0;
    int k = 0, row = 0, tries = 0;
    bool converged = false;
    while (k < kmax && tries < m2) {
        tries++;
        // row `row` of the residual: B(row, :) - sum_l U_l(row) V_l
        const int iv = A.perm[B.r0 + (row % B.m)], c = row / B.m;
        float2 *vk = V + (int64_t)k * n2;
        // the row from the column of iv over the trial cluster (B11, B22
        // symmetric, B12(i, j) = -B21(j, i)); rows and columns of the phi
        // component scaled by alpha
        {
            const float sr = c ? alpha : 1.0f;
            cluster_column<CK0, CK1, MULTI>(
                A, B.cc, B.n, iv, Q, etab, [&](int p, int blk, float2 v) {
                    // v = block blk = 2 c' + d' of B(j, iv): entry (c, d) of the row
                    // is block (d, c) of the column, negated off the diagonal
                    const int cc_ = blk >> 1, dd = blk & 1;   // column block (c', d')
                    if (dd != c) return;                      // need d' = c
                    const float f = (cc_ == c ? 1.0f : -1.0f) * sr * (cc_ ? alpha : 1.0f);
                    vk[cc_ * B.n + p] = make_float2(f * v.x, f * v.y);
                });
        }
        float best = -1.0f;
        int bidx = -1;
        for (int q = threadIdx.x; q < n2; q += ACA_THREADS) {
            float2 r = vk[q];
            for (int l = 0; l < k; l++) {
                const float2 p = cmulf(U[(int64_t)l * m2 + row], V[(int64_t)l * n2 + q]);
                r.x -= p.x;
                r.y -= p.y;
            }
            vk[q] = r;
            const float a = r.x * r.x + r.y * r.y;
            if (a > best || (a == best && bidx >= 0 && q < bidx)) {
                best = a;
                bidx = q;
            }
        }
        __syncthreads();
        float pv;
        int pj;
        block_argmax(best, bidx, rv, ri, pv, pj);
        if (threadIdx.x == 0) used[row] = 1;
        __syncthreads();
        if (!(pv > 0.0f) || pj < 0) {
            // zero residual row: take the next unused row
            int nxt = -1;
            for (int r = 0; r < m2; r++)
                if (!used[r]) {
                    nxt = r;
                    break;
                }
            if (nxt < 0) {
                converged = true;
                break;
            }
            row = nxt;
            continue;
        }
        // v = residual row / pivot
        const float2 piv = vk[pj];
        const float inv = 1.0f / (piv.x * piv.x + piv.y * piv.y);
        const float2 ipiv = make_float2(piv.x * inv, -piv.y * inv);
        __syncthreads();
        for (int q = threadIdx.x; q < n2; q += ACA_THREADS) vk[q] = cmulf(vk[q], ipiv);
        // column pj of the residual: B(:, pj) - sum_l V_l(pj) U_l
        const int jv = A.perm[B.c0 + (pj % B.n)], d = pj / B.n;
        float2 *uk = U + (int64_t)k * m2;
        {
            const float sc = d ? alpha : 1.0f;
            cluster_column<CK0, CK1, MULTI>(A, B.rc, B.m, jv, Q, etab,
                                            [&](int p, int blk, float2 v) {
                const int c_ = blk >> 1, dd = blk & 1;
                if (dd != d) return;
                const float f = sc * (c_ ? alpha : 1.0f);
                uk[c_ * B.m + p] = make_float2(f * v.x, f * v.y);
            });
        }
        for (int q = threadIdx.x; q < m2; q += ACA_THREADS) {
            float2 u = uk[q];
            for (int l = 0; l < k; l++) {
                const float2 p = cmulf(V[(int64_t)l * n2 + pj], U[(int64_t)l * m2 + q]);
                u.x -= p.x;
                u.y -= p.y;
            }
            uk[q] = u;
        }
        __syncthreads();
        // ||S_k||^2 = ||S_{k-1}||^2 + |u|^2 |v|^2 + 2 Re sum_l <u_k, u_l> <v_k, v_l>
        double uu = 0, vv = 0;
        for (int q = threadIdx.x; q < m2; q += ACA_THREADS)
            uu += (double)uk[q].x * uk[q].x + (double)uk[q].y * uk[q].y;
        for (int q = threadIdx.x; q < n2; q += ACA_THREADS)
            vv += (double)vk[q].x * vk[q].x + (double)vk[q].y * vk[q].y;
        uu = block_sum(uu, red);
        vv = block_sum(vv, red);
        double cross = 0.0;
        for (int l = 0; l < k; l++) {
            double ar = 0, ai = 0, br = 0, bi = 0;
            const float2 *ul = U + (int64_t)l * m2, *vl = V + (int64_t)l * n2;
            for (int q = threadIdx.x; q < m2; q += ACA_THREADS) {   // <u_k, u_l>
                ar += (double)uk[q].x * ul[q].x + (double)uk[q].y * ul[q].y;
                ai += (double)uk[q].y * ul[q].x - (double)uk[q].x * ul[q].y;
            }
            for (int q = threadIdx.x; q < n2; q += ACA_THREADS) {   // <v_k, v_l>
                br += (double)vk[q].x * vl[q].x + (double)vk[q].y * vl[q].y;
                bi += (double)vk[q].y * vl[q].x - (double)vk[q].x * vl[q].y;
            }
            ar = block_sum(ar, red);
            ai = block_sum(ai, red);
            br = block_sum(br, red);
            bi = block_sum(bi, red);
            cross += ar * br - ai * bi;
        }
        norm2 += uu * vv + 2.0 * cross;
        k++;
        if (uu * vv <= (double)tol * tol * norm2) {
            converged = true;
            break;
        }
        // next row: the largest |u_k| among the rows not used yet
        float bu = -1.0f;
        int bu_i = -1;
        for (int q = threadIdx.x; q < m2; q += ACA_THREADS) {
            if (used[q]) continue;
            const float a = uk[q].x * uk[q].x + uk[q].y * uk[q].y;
            if (a > bu || (a == bu && bu_i >= 0 && q < bu_i)) {
                bu = a;
                bu_i = q;
            }
        }
        float nv;
        int ni;
        block_argmax(bu, bu_i, rv, ri, nv, ni);
        if (ni < 0) {
            converged = true;
            break;
        }
        row = ni;
    }
    // every row tried: the cross approximation interpolates all rows (exact)
    if (!converged && k < kmax) converged = true;
    if (threadIdx.x == 0) rank[blockIdx.x] = converged ? k : kmax + 1;
}

// Dense leaf blocks: D_b [2n][2m] (column-major), entry (c m + i, d n + j) =
// B_far block (c, d) of (test vertex i, trial vertex j); grid (blocks, m n / 256).
struct NearBlock {
    int r0, m, c0, n;
    int rc;          // test leaf cluster
    int64_t off;
};

template <bool CK0, bool CK1, bool MULTI>
__global__ __launch_bounds__(ACA_THREADS) void near_dense_kernel(EntryArgs A,
                                                                 const NearBlock *blocks,
                                                                 float2 *D) {
    extern __shared__ double2 qs[];   // 12 values per triangle of the test leaf
    __shared__ double2 etab[256];
    const NearBlock B = blocks[blockIdx.x];
    const int jl = blockIdx.y;
    if (jl >= B.n) return;
    DM<double>::fill_table(etab);
    __syncthreads();
    float2 *d = D + B.off;
    const int64_t m2 = 2 * B.m;
    cluster_column<CK0, CK1, MULTI>(A, B.rc, B.m, A.perm[B.c0 + jl], qs, etab,
                                    [&](int p, int blk, float2 v) {
                                        const int c = blk >> 1, dd = blk & 1;
                                        d[(int64_t)(dd * B.n + jl) * m2 + c * B.m + p] = v;
                                    });
}

// compaction of the converged factors: U [r][2m], V [r][2n]
// (the scaling of the phi rows and columns by alpha undone)
__global__ __launch_bounds__(256) void aca_compact_kernel(const AcaBlock *blocks,
                                                          const int32_t *rank,
                                                          const int64_t *uo, const int64_t *vo,
                                                          const float2 *scr, float ialpha,
                                                          float2 *U, float2 *V) {
    const AcaBlock B = blocks[blockIdx.x];
    const int r = rank[blockIdx.x];
    const int64_t nu = (int64_t)r * 2 * B.m, nv = (int64_t)r * 2 * B.n;
    for (int64_t q = threadIdx.x; q < nu; q += 256) {
        const float2 a = scr[B.uoff + q];
        const float f = (q % (2 * B.m)) >= B.m ? ialpha : 1.0f;
        U[uo[blockIdx.x] + q] = make_float2(f * a.x, f * a.y);
    }
    for (int64_t q = threadIdx.x; q < nv; q += 256) {
        const float2 a = scr[B.voff + q];
        const float f = (q % (2 * B.n)) >= B.n ? ialpha : 1.0f;
        V[vo[blockIdx.x] + q] = make_float2(f * a.x, f * a.y);
    }
}

// The four blocks of B_far at sampled vertex pairs (scaling of the ACA).
template <bool CK0, bool CK1, bool MULTI>
__global__ __launch_bounds__(256) void sample_entries_kernel(EntryArgs A, const int2 *pairs,
                                                             int n, float2 *out) {
    __shared__ double2 etab[256];
    DM<double>::fill_table(etab);
    __syncthreads();
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    float2 e[4];
    vertex_entries<CK0, CK1, MULTI>(A, pairs[k].x, pairs[k].y, etab, e);
    for (int b = 0; b < 4; b++) out[4 * k + b] = e[b];
}

// x (complex128, original order) -> xt [2][N] complex64 in tree order
__global__ __launch_bounds__(256) void hmat_gather_kernel(const double2 *__restrict__ x,
                                                          const int32_t *__restrict__ perm,
                                                          int64_t N, float2 *__restrict__ xt) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= N) return;
    const int v = perm[p];
    xt[p] = make_float2((float)x[v].x, (float)x[v].y);
    xt[N + p] = make_float2((float)x[N + v].x, (float)x[N + v].y);
}

// z_b = V_b^T x_sigma (one workgroup per block; a wavefront per rank index)
struct LrBlock {
    int r0, m, c0, n, rank;
    int64_t uoff, voff, zoff;
};

__global__ __launch_bounds__(256) void hmat_z_kernel(const LrBlock *blocks, const float2 *V,
                                                     const float2 *__restrict__ xt, int64_t N,
                                                     double2 *z) {
    const LrBlock B = blocks[blockIdx.x];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n2 = 2 * B.n;
    for (int l = wave; l < B.rank; l += 4) {
        const float2 *v = V + B.voff + (int64_t)l * n2;
        double sr = 0, si = 0;
        for (int q = lane; q < n2; q += 64) {
            const int d = q >= B.n ? 1 : 0;
            const float2 a = v[q], b = xt[d * N + B.c0 + q - d * B.n];
            sr += (double)a.x * b.x - (double)a.y * b.y;
            si += (double)a.x * b.y + (double)a.y * b.x;
        }
        for (int o = 32; o > 0; o >>= 1) {
            sr += __shfl_xor(sr, o, 64);
            si += __shfl_xor(si, o, 64);
        }
        if (lane == 0) z[B.zoff + l] = make_double2(sr, si);
    }
}

// Rows of one test leaf: y = sum over the admissible blocks of its ancestors
// (root first) of U_b z_b + sum over its dense blocks of D_b x_sigma, written
// in the original vertex order.
__global__ __launch_bounds__(ROW_THREADS) void hmat_rows_kernel(
    const int32_t *__restrict__ leaf_v0, const int32_t *__restrict__ leaf_m,
    const int32_t *__restrict__ lb_ptr, const int32_t *__restrict__ lb_idx,
    const int32_t *__restrict__ ln_ptr, const int32_t *__restrict__ ln_idx,
    const LrBlock *__restrict__ lr, const float2 *__restrict__ U, const double2 *__restrict__ z,
    const NearBlock *__restrict__ nb, const float2 *__restrict__ D,
    const float2 *__restrict__ xt, const int32_t *__restrict__ perm, int64_t N,
    double2 *__restrict__ yf) {
    const int lf = blockIdx.x;
    const int v0 = leaf_v0[lf], m = leaf_m[lf];
    const int t = threadIdx.x;
    if (t >= 2 * m) return;
    const int c = t >= m ? 1 : 0, i = t - c * m;
    double sr = 0, si = 0;
    for (int e = lb_ptr[lf]; e < lb_ptr[lf + 1]; e++) {
        const LrBlock B = lr[lb_idx[e]];
        const int row = c * B.m + (v0 + i - B.r0);
        const float2 *u = U + B.uoff + row;
        const int64_t m2 = 2 * B.m;
        for (int l = 0; l < B.rank; l++) {
            const float2 a = u[l * m2];
            const double2 b = z[B.zoff + l];
            sr += a.x * b.x - a.y * b.y;
            si += a.x * b.y + a.y * b.x;
        }
    }
    for (int e = ln_ptr[lf]; e < ln_ptr[lf + 1]; e++) {
        const NearBlock B = nb[ln_idx[e]];
        const int64_t m2 = 2 * B.m;
        const float2 *d = D + B.off + c * B.m + i;
        for (int q = 0; q < 2 * B.n; q++) {
            const int dd = q >= B.n ? 1 : 0;
            const float2 a = d[q * m2], b = xt[dd * N + B.c0 + q - dd * B.n];
            sr += (double)a.x * b.x - (double)a.y * b.y;
            si += (double)a.x * b.y + (double)a.y * b.x;
        }
    }
    yf[c * N + perm[v0 + i]] = make_double2(sr, si);
}

// y = yf + near-field CSR x (FP64)
__global__ __launch_bounds__(256) void hmat_finish_kernel(
    const double2 *__restrict__ yf, const int32_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const double2 *__restrict__ nf, int64_t nnz,
    const double2 *__restrict__ x, int64_t N, double2 *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    double y1r = yf[i].x, y1i = yf[i].y, y2r = yf[N + i].x, y2i = yf[N + i].y;
    const double2 *C11 = nf, *C12 = nf + nnz, *C21 = nf + 2 * nnz, *C22 = nf + 3 * nnz;
    for (int e = rowptr[i]; e < rowptr[i + 1]; e++) {
        const int j = col[e];
        const double2 p = x[j], f = x[N + j];
        const double2 a = C11[e], b = C12[e], c = C21[e], d = C22[e];
        y1r += a.x * p.x - a.y * p.y + b.x * f.x - b.y * f.y;
        y1i += a.x * p.y + a.y * p.x + b.x * f.y + b.y * f.x;
        y2r += c.x * p.x - c.y * p.y + d.x * f.x - d.y * f.y;
        y2i += c.x * p.y + c.y * p.x + d.x * f.y + d.y * f.x;
    }
    y[i] = make_double2(y1r, y1i);
    y[N + i] = make_double2(y2r, y2i);
}

template <bool A_, bool B_, bool C_>
void launch_aca(int nb, EntryArgs ea, const AcaBlock *blocks, int kmax, float tol, float alpha,
                float2 *scr, int32_t *used, int32_t *rank, hipStream_t s) {
    hipLaunchKernelGGL((aca_kernel<A_, B_, C_>), dim3(nb), dim3(ACA_THREADS), 0, s, ea, blocks,
                       kmax, tol, alpha, scr, used, rank);
}
template <bool A_, bool B_, bool C_>
void launch_sample(int n, EntryArgs ea, const int2 *pairs, float2 *out, hipStream_t s) {
    hipLaunchKernelGGL((sample_entries_kernel<A_, B_, C_>), dim3((n + 255) / 256), dim3(256), 0, s,
                       ea, pairs, n, out);
}
template <bool A_, bool B_, bool C_>
void launch_near(int nb, int gy, size_t lds, EntryArgs ea, const NearBlock *blocks, float2 *D,
                 hipStream_t s) {
    hipLaunchKernelGGL((near_dense_kernel<A_, B_, C_>), dim3(nb, gy), dim3(ACA_THREADS), lds, s,
                       ea, blocks, D);
}

}   // namespace

// Compressed operator (cached per wavenumber pair and materials).
struct HMatrix {
    int64_t N = 0;
    HMatStats st{};
    DevBuf<int32_t> perm;                 // tree position -> vertex
    DevBuf<LrBlock> lr;
    DevBuf<float2> U, V;
    DevBuf<NearBlock> nb;
    DevBuf<float2> D;
    DevBuf<int32_t> leaf_v0, leaf_m, lb_ptr, lb_idx, ln_ptr, ln_idx;
    int nleaves = 0, nlr = 0;
    int64_t zlen = 0;
    DevBuf<double2> z, yf;
    DevBuf<float2> xt;
    int64_t bytes() const {
        return perm.bytes() + lr.bytes() + U.bytes() + V.bytes() + nb.bytes() + D.bytes() +
               leaf_v0.bytes() + leaf_m.bytes() + lb_ptr.bytes() + lb_idx.bytes() +
               ln_ptr.bytes() + ln_idx.bytes() + z.bytes() + yf.bytes() + xt.bytes();
    }
};

void HMatDeleter::operator()(HMatrix *p) const { delete p; }
int64_t hmat_bytes(const HMatrix &h) { return h.bytes(); }
const HMatStats &hmat_stats(const HMatrix &h) { return h.st; }

std::unique_ptr<HMatrix, HMatDeleter> hmat_build(bem_mesh *m, const NearOperator &nf, double2 k0,
                                                 hipStream_t s) {
    const auto t_start = std::chrono::steady_clock::now();
    const Tuning &tn = tuning();
    const int leaf = tn.hmat_leaf.load();
    const double eta = tn.hmat_eta_pct.load() / 100.0;
    const float tol = (float)(tn.hmat_tol_ppb.load() * 1e-9);
    const int kmax = tn.hmat_kmax.load();
    std::unique_ptr<HMatrix, HMatDeleter> H(new HMatrix());
    const int64_t N = m->N;
    H->N = N;
    // per vertex: the box of its star's triangles
    TreeBuilder tb;
    tb.m = m;
    tb.leaf = leaf;
    tb.tlo.assign(3 * N, 1e300);
    tb.thi.assign(3 * N, -1e300);
    for (int64_t t = 0; t < m->T; t++)
        for (int a = 0; a < 3; a++) {
            const int v = m->tri[3 * t + a];
            for (int b = 0; b < 3; b++) {
                const int w = m->tri[3 * t + b];
                for (int c = 0; c < 3; c++) {
                    tb.tlo[3 * v + c] = std::min(tb.tlo[3 * v + c], m->P[3 * w + c]);
                    tb.thi[3 * v + c] = std::max(tb.thi[3 * v + c], m->P[3 * w + c]);
                }
            }
        }
    tb.order.resize(N);
    std::iota(tb.order.begin(), tb.order.end(), 0);
    tb.build(0, (int)N, -1);
    const std::vector<Cluster> &cl = tb.cl;
    BlockLists bl;
    build_blocks(cl, 0, 0, eta, bl);
    H->perm.upload(tb.order);

    // per cluster: its triangles (sorted) and each vertex's slots in that list
    std::vector<std::vector<std::pair<int32_t, int32_t>>> star(N);   // vertex -> (tri, a)
    for (int64_t t = 0; t < m->T; t++)
        for (int a = 0; a < 3; a++) star[m->tri[3 * t + a]].push_back({(int32_t)t, a});
    const int ncl = (int)cl.size();
    std::vector<int32_t> ct_ptr(ncl + 1, 0), ct_idx, cv_ptr, cv_slot;
    std::vector<int64_t> cv_off(ncl);
    std::vector<int32_t> ntri(ncl);
    for (int c = 0; c < ncl; c++) {
        std::vector<int32_t> ts;
        for (int p = cl[c].v0; p < cl[c].v1; p++)
            for (const auto &ta : star[tb.order[p]]) ts.push_back(ta.first);
        std::sort(ts.begin(), ts.end());
        ts.erase(std::unique(ts.begin(), ts.end()), ts.end());
        ntri[c] = (int32_t)ts.size();
        cv_off[c] = (int64_t)cv_ptr.size();
        cv_ptr.push_back((int32_t)cv_slot.size());
        for (int p = cl[c].v0; p < cl[c].v1; p++) {
            for (const auto &ta : star[tb.order[p]]) {
                const int k = (int)(std::lower_bound(ts.begin(), ts.end(), ta.first) - ts.begin());
                cv_slot.push_back(3 * k + ta.second);
            }
            cv_ptr.push_back((int32_t)cv_slot.size());
        }
        ct_idx.insert(ct_idx.end(), ts.begin(), ts.end());
        ct_ptr[c + 1] = (int32_t)ct_idx.size();
    }
    DevBuf<int32_t> ct_ptr_d, ct_idx_d, cv_ptr_d, cv_slot_d;
    DevBuf<int64_t> cv_off_d;
    ct_ptr_d.upload(ct_ptr);
    ct_idx_d.upload(ct_idx);
    cv_off_d.upload(cv_off);
    cv_ptr_d.upload(cv_ptr);
    cv_slot_d.upload(cv_slot);

    // entry arguments
    EntryArgs ea;
    ea.geo = m->geo64.p;
    ea.tst = m->tst.p;
    ea.tobj = m->tobj_d.p;
    ea.tri = m->tri_d.p;
    ea.star_ptr = m->star_ptr.p;
    ea.star_idx = m->star_idx.p;
    ea.perm = H->perm.p;
    ea.cf = make_dcoef<double>(k0, nf);
    DevBuf<double> itab;
    if (m->nobj > 1) {
        constexpr size_t W = sizeof(DIntT<double>) / sizeof(double);
        std::vector<double> h((size_t)m->nobj * W);
        for (int o = 0; o < m->nobj; o++) {
            const DIntT<double> c = make_dint<double>(k0, nf.k1o[o], nf.rhoo[o], nf.s1);
            std::memcpy(h.data() + (size_t)o * W, &c, sizeof(c));
        }
        itab.upload(h);
    }
    ea.itab = (const DIntT<double> *)itab.p;
    ea.ct_ptr = ct_ptr_d.p;
    ea.ct_idx = ct_idx_d.p;
    ea.cv_off = cv_off_d.p;
    ea.cv_ptr = cv_ptr_d.p;
    ea.cv_slot = cv_slot_d.p;
    const int code = variant_code(m, k0, nf);

    // Scaling of the phi rows and columns, alpha = sqrt(rms B11 / rms B22) over
    // one vertex pair of each admissible block (up to 4096): the hypersingular
    // block is about k^2 larger than the single layer, and the cross
    // approximation's tolerance is relative to the whole block.
    float alpha = 1.0f;
    if (!bl.adm.empty()) {
        std::vector<int2> pairs;
        const int stride = std::max<int>(1, (int)bl.adm.size() / 4096);
        for (size_t b = 0; b < bl.adm.size(); b += stride) {
            const Cluster &A = cl[bl.adm[b].first], &B = cl[bl.adm[b].second];
            pairs.push_back(make_int2(tb.order[(A.v0 + A.v1) / 2], tb.order[(B.v0 + B.v1) / 2]));
        }
        const int np_ = (int)pairs.size();
        DevBuf<int2> pd;
        pd.upload(pairs);
        DevBuf<float2> od((size_t)4 * np_);
        switch (code) {
        case 0: launch_sample<false, false, false>(np_, ea, pd.p, od.p, s); break;
        case 1: launch_sample<false, false, true>(np_, ea, pd.p, od.p, s); break;
        case 2: launch_sample<false, true, false>(np_, ea, pd.p, od.p, s); break;
        case 3: launch_sample<false, true, true>(np_, ea, pd.p, od.p, s); break;
        case 4: launch_sample<true, false, false>(np_, ea, pd.p, od.p, s); break;
        case 5: launch_sample<true, false, true>(np_, ea, pd.p, od.p, s); break;
        case 6: launch_sample<true, true, false>(np_, ea, pd.p, od.p, s); break;
        default: launch_sample<true, true, true>(np_, ea, pd.p, od.p, s); break;
        }
        BEM_LAUNCH_CHECK();
        std::vector<float2> e((size_t)4 * np_);
        BEM_HIP(hipMemcpyAsync(e.data(), od.p, e.size() * sizeof(float2), hipMemcpyDeviceToHost, s));
        BEM_HIP(hipStreamSynchronize(s));
        double s11 = 0, s22 = 0;
        for (int k = 0; k < np_; k++) {
            s11 += (double)e[4 * k].x * e[4 * k].x + (double)e[4 * k].y * e[4 * k].y;
            s22 += (double)e[4 * k + 3].x * e[4 * k + 3].x + (double)e[4 * k + 3].y * e[4 * k + 3].y;
        }
        if (s11 > 0 && s22 > 0 && std::isfinite(s11 / s22))
            alpha = (float)std::pow(s11 / s22, 0.25);
    }
    H->st.alpha = alpha;

    // ACA over the admissible blocks, in batches bounded by the scratch size.
    // A block whose cross approximation has not reached the tolerance after
    // kmax terms is replaced by the pairs of its children (leaf pairs become
    // dense blocks) and those are approximated in the next round.
    std::vector<AcaBlock> ab;      // converged blocks (uoff/voff into H->U, H->V)
    std::vector<int32_t> rank;
    std::vector<std::pair<int, int>> pending = bl.adm, kept;
    const int64_t scr_cap = (int64_t)1 << 28;   // float2 entries per batch (2 GiB)
    struct Chunk {
        int64_t u0 = 0, v0 = 0;   // place of the chunk in U, V
        DevBuf<float2> U, V;
    };
    std::vector<Chunk> chunks;
    int64_t u_total = 0, v_total = 0;
    while (!pending.empty()) {
        std::vector<std::pair<int, int>> next;
        const int np_ = (int)pending.size();
        int b0 = 0;
        while (b0 < np_) {
            std::vector<AcaBlock> batch;
            int64_t off = 0, used_off = 0;
            int b1 = b0;
            while (b1 < np_) {
                const Cluster &A = cl[pending[b1].first], &B = cl[pending[b1].second];
                const int64_t mm = A.v1 - A.v0, nn = B.v1 - B.v0;
                // 12 complex128 values (24 float2 slots) per triangle
                const int64_t nq =
                    24 * (int64_t)std::max(ntri[pending[b1].first], ntri[pending[b1].second]);
                const int64_t need = (int64_t)kmax * 2 * (mm + nn) + nq;
                if (b1 > b0 && off + need > scr_cap) break;
                AcaBlock q;
                q.r0 = A.v0;
                q.m = (int)mm;
                q.c0 = B.v0;
                q.n = (int)nn;
                q.rc = pending[b1].first;
                q.cc = pending[b1].second;
                q.uoff = off;
                q.voff = off + (int64_t)kmax * 2 * mm;
                q.qoff = q.voff + (int64_t)kmax * 2 * nn;
                q.used_off = used_off;
                batch.push_back(q);
                off += need;
                used_off += 2 * mm;
                b1++;
            }
            const int cnt = b1 - b0;
            DevBuf<AcaBlock> blocks_d;
            blocks_d.upload(batch);
            DevBuf<float2> scr((size_t)off);
            DevBuf<int32_t> used((size_t)used_off), rank_d((size_t)cnt);
            switch (code) {
            case 0: launch_aca<false, false, false>(cnt, ea, blocks_d.p, kmax, tol, alpha, scr.p, used.p, rank_d.p, s); break;
            case 1: launch_aca<false, false, true>(cnt, ea, blocks_d.p, kmax, tol, alpha, scr.p, used.p, rank_d.p, s); break;
            case 2: launch_aca<false, true, false>(cnt, ea, blocks_d.p, kmax, tol, alpha, scr.p, used.p, rank_d.p, s); break;
            case 3: launch_aca<false, true, true>(cnt, ea, blocks_d.p, kmax, tol, alpha, scr.p, used.p, rank_d.p, s); break;
            case 4: launch_aca<true, false, false>(cnt, ea, blocks_d.p, kmax, tol, alpha, scr.p, used.p, rank_d.p, s); break;
            case 5: launch_aca<true, false, true>(cnt, ea, blocks_d.p, kmax, tol, alpha, scr.p, used.p, rank_d.p, s); break;
            case 6: launch_aca<true, true, false>(cnt, ea, blocks_d.p, kmax, tol, alpha, scr.p, used.p, rank_d.p, s); break;
            default: launch_aca<true, true, true>(cnt, ea, blocks_d.p, kmax, tol, alpha, scr.p, used.p, rank_d.p, s); break;
            }
            BEM_LAUNCH_CHECK();
            std::vector<int32_t> rk(cnt);
            BEM_HIP(hipMemcpyAsync(rk.data(), rank_d.p, cnt * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, s));
            BEM_HIP(hipStreamSynchronize(s));
            // converged blocks are copied to a compact chunk of factors (rank 0
            // for the others, which are split); chunks are joined at the end
            std::vector<int64_t> uo(cnt), vo(cnt);
            int64_t ut = 0, vt = 0;
            const int64_t u_old = u_total, v_old = v_total;
            for (int q = 0; q < cnt; q++) {
                const std::pair<int, int> pr = pending[b0 + q];
                if (rk[q] > kmax) {
                    H->st.split_blocks++;
                    const Cluster &A = cl[pr.first], &B = cl[pr.second];
                    const bool la = A.child[0] < 0, lb = B.child[0] < 0;
                    if (la && lb) {
                        bl.nearb.push_back(pr);
                    } else if (la) {
                        for (int c : B.child) next.push_back({pr.first, c});
                    } else if (lb) {
                        for (int c : A.child) next.push_back({c, pr.second});
                    } else {
                        for (int a : A.child)
                            for (int c : B.child) next.push_back({a, c});
                    }
                    rk[q] = 0;
                    uo[q] = vo[q] = 0;
                    continue;
                }
                uo[q] = u_old + ut;
                vo[q] = v_old + vt;
                ut += (int64_t)rk[q] * 2 * batch[q].m;
                vt += (int64_t)rk[q] * 2 * batch[q].n;
                AcaBlock kb = batch[q];
                kb.uoff = uo[q];
                kb.voff = vo[q];
                ab.push_back(kb);
                rank.push_back(rk[q]);
                kept.push_back(pr);
            }
            if (ut + vt > 0) {
                BEM_HIP(hipMemcpyAsync(rank_d.p, rk.data(), cnt * sizeof(int32_t),
                                       hipMemcpyHostToDevice, s));
                Chunk ch;
                ch.u0 = u_old;
                ch.v0 = v_old;
                ch.U.alloc((size_t)ut);
                ch.V.alloc((size_t)vt);
                // offsets within the chunk
                std::vector<int64_t> uc(cnt), vc(cnt);
                for (int q = 0; q < cnt; q++) {
                    uc[q] = rk[q] ? uo[q] - u_old : 0;
                    vc[q] = rk[q] ? vo[q] - v_old : 0;
                }
                DevBuf<int64_t> uo_d, vo_d;
                uo_d.upload(uc);
                vo_d.upload(vc);
                hipLaunchKernelGGL(aca_compact_kernel, dim3(cnt), dim3(256), 0, s, blocks_d.p,
                                   rank_d.p, uo_d.p, vo_d.p, scr.p, 1.0f / alpha, ch.U.p, ch.V.p);
                BEM_LAUNCH_CHECK();
                BEM_HIP(hipStreamSynchronize(s));
                chunks.push_back(std::move(ch));
                u_total += ut;
                v_total += vt;
            }
            b0 = b1;
        }
        pending.swap(next);
    }
    bl.adm = kept;
    const int na = (int)ab.size();
    H->U.alloc((size_t)std::max<int64_t>(u_total, 1));
    H->V.alloc((size_t)std::max<int64_t>(v_total, 1));
    for (Chunk &ch : chunks) {
        BEM_HIP(hipMemcpyAsync(H->U.p + ch.u0, ch.U.p, ch.U.bytes(), hipMemcpyDeviceToDevice, s));
        BEM_HIP(hipMemcpyAsync(H->V.p + ch.v0, ch.V.p, ch.V.bytes(), hipMemcpyDeviceToDevice, s));
    }
    BEM_HIP(hipStreamSynchronize(s));
    chunks.clear();
    // low-rank block table
    std::vector<LrBlock> lr(na);
    int64_t zoff = 0;
    int maxr = 0;
    double sumr = 0;
    for (int b = 0; b < na; b++) {
        lr[b] = LrBlock{ab[b].r0, ab[b].m, ab[b].c0, ab[b].n, rank[b], ab[b].uoff, ab[b].voff, zoff};
        zoff += rank[b];
        maxr = std::max(maxr, rank[b]);
        sumr += rank[b];
    }
    H->lr.upload(lr);
    H->nlr = na;
    H->zlen = std::max<int64_t>(zoff, 1);

    // dense leaf blocks
    const int nn_ = (int)bl.nearb.size();
    std::vector<NearBlock> nbh(nn_);
    int64_t doff = 0, maxn = 0, maxt = 0;
    for (int b = 0; b < nn_; b++) {
        const Cluster &A = cl[bl.nearb[b].first], &B = cl[bl.nearb[b].second];
        nbh[b] = NearBlock{A.v0, A.v1 - A.v0, B.v0, B.v1 - B.v0, bl.nearb[b].first, doff};
        doff += 4 * (int64_t)nbh[b].m * nbh[b].n;
        maxn = std::max<int64_t>(maxn, nbh[b].n);
        maxt = std::max<int64_t>(maxt, ntri[bl.nearb[b].first]);
    }
    {
        // blocks that did not converge at rank kmax end as dense leaf pairs:
        // report that instead of an allocation failure
        size_t fr = 0, tot = 0;
        BEM_HIP(hipMemGetInfo(&fr, &tot));
        const size_t need = (size_t)doff * sizeof(float2);
        if (need > fr)
            fail(BEM_E_NOMEM, "compressed operator: dense leaf blocks need " +
                                  std::to_string(need) + " bytes (" + std::to_string(nn_) +
                                  " leaf pairs, " + std::to_string(H->st.split_blocks) +
                                  " blocks split after not converging at rank " +
                                  std::to_string(kmax) + "), " + std::to_string(fr) +
                                  " bytes free");
    }
    H->nb.upload(nbh);
    H->D.alloc((size_t)std::max<int64_t>(doff, 1));
    if (nn_ > 0) {
        const int gy = (int)maxn;
        const size_t lds = (size_t)12 * maxt * sizeof(double2);
        if (lds > 65536 - 256 * sizeof(double2))
            fail(BEM_E_UNSUPPORTED, "leaf cluster with too many triangles");
        switch (code) {
        case 0: launch_near<false, false, false>(nn_, gy, lds, ea, H->nb.p, H->D.p, s); break;
        case 1: launch_near<false, false, true>(nn_, gy, lds, ea, H->nb.p, H->D.p, s); break;
        case 2: launch_near<false, true, false>(nn_, gy, lds, ea, H->nb.p, H->D.p, s); break;
        case 3: launch_near<false, true, true>(nn_, gy, lds, ea, H->nb.p, H->D.p, s); break;
        case 4: launch_near<true, false, false>(nn_, gy, lds, ea, H->nb.p, H->D.p, s); break;
        case 5: launch_near<true, false, true>(nn_, gy, lds, ea, H->nb.p, H->D.p, s); break;
        case 6: launch_near<true, true, false>(nn_, gy, lds, ea, H->nb.p, H->D.p, s); break;
        default: launch_near<true, true, true>(nn_, gy, lds, ea, H->nb.p, H->D.p, s); break;
        }
        BEM_LAUNCH_CHECK();
    }

    // per test leaf: admissible blocks of its ancestors (root first), dense blocks
    std::vector<std::vector<int32_t>> rows_of(cl.size()), near_of(cl.size());
    for (int b = 0; b < na; b++) rows_of[bl.adm[b].first].push_back(b);
    for (int b = 0; b < nn_; b++) near_of[bl.nearb[b].first].push_back(b);
    std::vector<int32_t> lv0, lm, lbp{0}, lbi, lnp{0}, lni;
    for (int c = 0; c < (int)cl.size(); c++) {
        if (cl[c].child[0] >= 0) continue;
        std::vector<int> path;
        for (int a = c; a >= 0; a = cl[a].parent) path.push_back(a);
        std::reverse(path.begin(), path.end());
        for (int a : path) lbi.insert(lbi.end(), rows_of[a].begin(), rows_of[a].end());
        lbp.push_back((int32_t)lbi.size());
        lni.insert(lni.end(), near_of[c].begin(), near_of[c].end());
        lnp.push_back((int32_t)lni.size());
        lv0.push_back(cl[c].v0);
        lm.push_back(cl[c].v1 - cl[c].v0);
    }
    H->nleaves = (int)lv0.size();
    H->leaf_v0.upload(lv0);
    H->leaf_m.upload(lm);
    H->lb_ptr.upload(lbp);
    H->lb_idx.upload(lbi.empty() ? std::vector<int32_t>{0} : lbi);
    H->ln_ptr.upload(lnp);
    H->ln_idx.upload(lni.empty() ? std::vector<int32_t>{0} : lni);
    H->z.alloc((size_t)H->zlen);
    H->yf.alloc((size_t)(2 * N));
    H->xt.alloc((size_t)(2 * N));
    BEM_HIP(hipStreamSynchronize(s));

    HMatStats &st = H->st;
    st.n_admissible = na;
    st.n_dense = nn_;
    st.max_rank = maxr;
    st.mean_rank = na ? sumr / na : 0.0;
    st.lowrank_bytes = (int64_t)(H->U.bytes() + H->V.bytes());
    st.dense_bytes = (int64_t)H->D.bytes();
    st.bytes = H->bytes();
    st.leaf = leaf;
    st.eta = eta;
    st.tol = tol;
    st.kmax = kmax;
    st.n_clusters = (int)cl.size();
    // fraction of the 4 N^2 entries held in low-rank and dense blocks
    double cover = 0;
    for (int b = 0; b < na; b++) cover += 4.0 * ab[b].m * (double)ab[b].n;
    st.admissible_fraction = cover / (4.0 * (double)N * (double)N);
    st.setup_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return H;
}

int64_t hmat_bytes_estimate(const bem_mesh *m, double2 k0, double2 k1, double rho) {
    auto it = m->hmat_cache.find(near_key(m, k0, k1, rho, 1, nullptr));
    if (it != m->hmat_cache.end()) return hmat_bytes(*it->second);
    return std::max<int64_t>(dense_bytes(m) / 4, (int64_t)1 << 30);
}

HMatrix &hmat_get(bem_mesh *m, double2 k0, double2 k1, double rho, hipStream_t s, int s1,
                  const ObjMaterials *om) {
    const NearKey key = near_key(m, k0, k1, rho, s1, om);
    auto it = m->hmat_cache.find(key);
    if (it != m->hmat_cache.end()) return *it->second;
    const NearOperator &nf = nearfield_get(m, k0, k1, rho, s, s1, om);
    if (m->hmat_cache.size() >= 2) m->hmat_cache.erase(m->hmat_cache.begin());
    auto h = hmat_build(m, nf, k0, s);
    HMatrix &ref = *h;
    m->hmat_cache.emplace(key, std::move(h));
    return ref;
}

void hmat_apply(HMatrix &H, bem_mesh *m, const NearOperator &nf, const double2 *x, double2 *y,
                hipStream_t s) {
    Timer tm("hmat_apply", s);
    const int64_t N = H.N;
    hipLaunchKernelGGL(hmat_gather_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, x,
                       H.perm.p, N, H.xt.p);
    if (H.nlr > 0)
        hipLaunchKernelGGL(hmat_z_kernel, dim3(H.nlr), dim3(256), 0, s, H.lr.p, H.V.p, H.xt.p, N,
                           H.z.p);
    hipLaunchKernelGGL(hmat_rows_kernel, dim3(H.nleaves), dim3(ROW_THREADS), 0, s, H.leaf_v0.p,
                       H.leaf_m.p, H.lb_ptr.p, H.lb_idx.p, H.ln_ptr.p, H.ln_idx.p, H.lr.p, H.U.p,
                       H.z.p, H.nb.p, H.D.p, H.xt.p, H.perm.p, N, H.yf.p);
    hipLaunchKernelGGL(hmat_finish_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                       H.yf.p, m->nf_rowptr.p, m->nf_col.p, (const double2 *)nf.vals.p,
                       m->nf_nnz, x, N, y);
    BEM_LAUNCH_CHECK();
}

}   // namespace bem

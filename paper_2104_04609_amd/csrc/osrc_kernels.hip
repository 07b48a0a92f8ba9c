// Device kernels of the OSRC preconditioner: batched block-LDL^T solves over
// the nested-dissection tree (all shifted systems share one pattern) and the
// elementwise Pade partial-fraction sums.
#include <algorithm>
#include <mutex>

#include "osrc_internal.h"

namespace bem {

namespace {

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// threads of the one-launch level kernel: 1024 (64 rows of a block per
// pass) for batches of fewer than LVL_WIDE_MAX_RHS vectors, else 256
constexpr int LVL_WIDE_MAX_RHS = 4;
// levels with at least this many dissection blocks use the one-launch form
constexpr int LVL_FUSE_MIN_BLOCKS = 16;

// Block-LDL^T solve over the nested-dissection tree, one launch per level.
// Rows of a dissection block only reference rows of the same block or of its
// dissection descendants (forward) / ancestors (backward), which earlier
// launches have finished.  Work of one system: y [n] (external updates),
// z [n] (block results), then the partial sums of the split solve.
//
// forward, block B = rows [s0, s0 + w):
//   y_j = in[perm[j]] - sum_{k < s0} L_jk z_k         (external update)
//   z_B = inv(L_BB) y_B                               (dense block inverse)
// backward (levels from the top down):
//   y_j = Dinv_j z_j - sum_{i >= s0 + w} L_ij z_i      (external update)
//   z_B = inv(L_BB)^T y_B;  out[perm[j]] = scale z_j
// The dense inverses are read by rows: inv(L_BB) row r at invL[r w ..] and
// inv(L_BB)^T row r at invLT[r w ..], lanes over consecutive columns.
__device__ inline SolveTask task_of(const TaskList &tasks, int y) {
    const int b = y % tasks.nbase, r = y / tasks.nbase;
    SolveTask t = tasks.t[b];
    t.in += r * tasks.in_stride;
    t.out += r * tasks.out_stride;
    t.work += r * tasks.work_stride;
    return t;
}

template <int W>
__device__ inline double2 lane_sum(double sx, double sy) {
    for (int o = W / 2; o > 0; o >>= 1) {
        sx += __shfl_xor(sx, o, W);
        sy += __shfl_xor(sy, o, W);
    }
    return make_double2(sx, sy);
}

// Row rr of the dense block product, lane `ln` of W lanes (partial sum):
// forward sum_{c <= rr} inv(L_BB)[rr][c] v_c, backward sum_{c >= rr}.
template <bool FWD, int W, class V>
__device__ inline double2 dense_row(const double2 *__restrict__ row, int rr, int w, int ln, V v) {
    double sx = 0.0, sy = 0.0;
    const int c0 = FWD ? 0 : rr, c1 = FWD ? rr + 1 : w;
#pragma unroll 4
    for (int c = c0 + ln; c < c1; c += W) {
        const double2 p = cmul(row[c], v(c));
        sx += p.x;
        sy += p.y;
    }
    return make_double2(sx, sy);
}

// External update: one wavefront per row of the level (fixed-order
// butterfly), grid (ceil(rows / 4), tasks), or with WIDE one workgroup per
// row (long rows: the four wavefronts' sums added in LDS in wave order),
// grid (rows, tasks); level rows [rb, re) of lrow.
template <bool FWD, bool WIDE>
__global__ __launch_bounds__(256) void ldl_ext_kernel(LdlDev L, TaskList tasks, int rb, int re) {
    const SolveTask t = task_of(tasks, blockIdx.y);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = WIDE ? rb + blockIdx.x : rb + blockIdx.x * 4 + wave;
    if (r >= re) return;   // uniform over the workgroup when WIDE
    const LdlRow d = L.lrowd[r];
    const int j = d.j;
    double2 *y = t.work, *z = t.work + L.n;
    // the row's own term first: it does not wait for the sum
    double2 base = make_double2(0.0, 0.0);
    if (threadIdx.x == (WIDE ? 0 : threadIdx.x & ~63))
        base = FWD ? t.in[d.perm] : cmul(L.Dinv[(int64_t)t.factor * L.n + j], z[j]);
    const double2 *val = (FWD ? L.Lcsr : L.Lcsc) + (int64_t)t.factor * L.nnz;
    const int32_t *idx = FWD ? L.Rj : L.Li;
    const int e0 = FWD ? d.fx : d.bx, e1 = FWD ? d.fy : d.by;
    const int lanes = WIDE ? 256 : 64, me = WIDE ? (int)threadIdx.x : lane;
    double sx = 0.0, sy = 0.0;
#pragma unroll 4
    for (int e = e0 + me; e < e1; e += lanes) {
        const double2 p = cmul(val[e], z[idx[e]]);
        sx += p.x;
        sy += p.y;
    }
    double2 acc = lane_sum<64>(sx, sy);
    if (WIDE) {
        __shared__ double2 part[4];
        if (lane == 0) part[wave] = acc;
        __syncthreads();
        if (threadIdx.x != 0) return;
        acc = make_double2((part[0].x + part[1].x) + (part[2].x + part[3].x),
                           (part[0].y + part[1].y) + (part[2].y + part[3].y));
    }
    if (lane == 0) y[j] = make_double2(base.x - acc.x, base.y - acc.y);
}

// Dense block products of a level: one wavefront per row (any block width),
// grid (ceil(rows / 4), tasks); y_B is complete (previous launch).
template <bool FWD>
__global__ __launch_bounds__(256) void ldl_dense_kernel(LdlDev L, TaskList tasks, int rb, int re) {
    const SolveTask t = task_of(tasks, blockIdx.y);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = rb + blockIdx.x * 4 + wave;
    if (r >= re) return;
    const LdlRow d = L.lrowd[r];
    const double2 *y = t.work;
    double2 *z = t.work + L.n;
    const double2 *row = (FWD ? L.invL : L.invLT) + (int64_t)t.factor * L.ndense + d.doff +
                         (int64_t)d.rr * d.w;
    const double2 p = dense_row<FWD, 64>(row, d.rr, d.w, lane, [&](int c) { return y[d.s0 + c]; });
    const double2 acc = lane_sum<64>(p.x, p.y);
    if (lane == 0) {
        z[d.j] = acc;
        if (!FWD) t.out[d.perm] = cmul(t.scale, acc);
    }
}

// One level of the sweep (levels of many small blocks): workgroup (block,
// task) forms the external updates of its rows (16 lanes per row, fixed
// butterfly; rows of finished levels only) into LDS, then the dense block
// product (16 lanes per row).  Blocks lblkd[bb + blockIdx.x].  The first
// pass's dense entries (up to 64 columns a row) are loaded before the
// external updates, since they do not depend on them.
constexpr int LVL_PREFETCH = 4;
template <bool FWD, int LVL_THREADS>
__global__ __launch_bounds__(LVL_THREADS) void ldl_level_kernel(LdlDev L, TaskList tasks, int bb) {
    __shared__ double2 tb[LDL_MAX_BLOCK];
    const SolveTask t = task_of(tasks, blockIdx.y);
    const int4 bd = L.lblkd[bb + blockIdx.x];
    const int s0 = bd.x, w = bd.y;
    double2 *z = t.work + L.n;
    const double2 *val = (FWD ? L.Lcsr : L.Lcsc) + (int64_t)t.factor * L.nnz;
    const int32_t *idx = FWD ? L.Rj : L.Li;
    const double2 *dense = (FWD ? L.invL : L.invLT) + (int64_t)t.factor * L.ndense + bd.z;
    const int grp = threadIdx.x >> 4, gl = threadIdx.x & 15;
    // dense entries of row grp, columns c0 + gl + 16 q (the order of dense_row)
    double2 pre[LVL_PREFETCH];
    {
        const int rr = grp, c0 = FWD ? 0 : rr, c1 = FWD ? rr + 1 : w;
#pragma unroll
        for (int q = 0; q < LVL_PREFETCH; q++) {
            const int c = c0 + gl + 16 * q;
            pre[q] = rr < w && c < c1 ? dense[(int64_t)rr * w + c] : make_double2(0.0, 0.0);
        }
    }
    int perm0 = 0;   // perm of row grp (first pass), for the backward output
    for (int r0 = 0; r0 < w; r0 += LVL_THREADS / 16) {
        const int r = r0 + grp;
        double sx = 0.0, sy = 0.0;
        double2 base = make_double2(0.0, 0.0);
        if (r < w) {
            const LdlRow d = L.jrow[s0 + r];
            if (r0 == 0) perm0 = d.perm;
            if (gl == 0)
                base = FWD ? t.in[d.perm]
                           : cmul(L.Dinv[(int64_t)t.factor * L.n + s0 + r], z[s0 + r]);
            const int e0 = FWD ? d.fx : d.bx, e1 = FWD ? d.fy : d.by;
#pragma unroll 4
            for (int e = e0 + gl; e < e1; e += 16) {
                const double2 p = cmul(val[e], z[idx[e]]);
                sx += p.x;
                sy += p.y;
            }
        }
        const double2 acc = lane_sum<16>(sx, sy);
        if (r < w && gl == 0) tb[r] = make_double2(base.x - acc.x, base.y - acc.y);
    }
    __syncthreads();
    for (int r0 = 0; r0 < w; r0 += LVL_THREADS / 16) {
        const int r = r0 + grp;
        double2 p = make_double2(0.0, 0.0);
        if (r < w) {
            const int c0 = FWD ? 0 : r, c1 = FWD ? r + 1 : w;
            if (r0 == 0 && c1 - c0 <= 16 * LVL_PREFETCH) {
                double sx = 0.0, sy = 0.0;
#pragma unroll
                for (int q = 0; q < LVL_PREFETCH; q++) {
                    const int c = c0 + gl + 16 * q;
                    if (c < c1) {
                        const double2 v = cmul(pre[q], tb[c]);
                        sx += v.x;
                        sy += v.y;
                    }
                }
                p = make_double2(sx, sy);
            } else {
                p = dense_row<FWD, 16>(dense + (int64_t)r * w, r, w, gl,
                                       [&](int c) { return tb[c]; });
            }
        }
        const double2 acc = lane_sum<16>(p.x, p.y);
        if (r < w && gl == 0) {
            z[s0 + r] = acc;
            if (!FWD) t.out[r0 == 0 ? perm0 : L.jrow[s0 + r].perm] = cmul(t.scale, acc);
        }
    }
}

// ------------------------------------------------ two-part (split) solve
// Bottom subtrees: one workgroup per (subtree, task) holds the subtree's rows
// in LDS (row j at j - r0) and runs its heights in order (forward) or in
// reverse (backward), an external update phase then a dense phase (16 lanes
// per row each, fixed butterflies).  The forward kernel also forms, for
// every top row, the partial sum of its external entries inside the subtree,
// unless the top part is solved by the level kernels.  The top part: one
// workgroup per task (forward, D^{-1}, backward) with its rows in LDS at
// their local index, or level by level through the global work vector.
constexpr int SPLIT_THREADS = 1024;

// Sum of 16 lanes (fixed butterfly; all 16 lanes of the group take part).
__device__ inline double2 sum16(double sx, double sy) {
    for (int o = 8; o > 0; o >>= 1) {
        sx += __shfl_xor(sx, o, 16);
        sy += __shfl_xor(sy, o, 16);
    }
    return make_double2(sx, sy);
}

// Sum over the lpr lanes of a group (lpr = 2, 4, 8 or 16, groups aligned to
// lpr lanes; fixed butterfly).
__device__ inline double2 group_sum(double sx, double sy, int lpr) {
    for (int o = lpr >> 1; o > 0; o >>= 1) {
        sx += __shfl_xor(sx, o, 16);
        sy += __shfl_xor(sy, o, 16);
    }
    return make_double2(sx, sy);
}

// Lanes per row for `cnt` rows in one pass of the workgroup where possible
// (fewer lanes per row, more rows at once: every pass costs a round trip).
__device__ inline int split_lanes(int cnt) {
    return cnt * 16 <= SPLIT_THREADS ? 16 : cnt * 8 <= SPLIT_THREADS ? 8
                                          : cnt * 4 <= SPLIT_THREADS ? 4 : 2;
}

// Dense phase on `cnt` rows: `row_of(k, loc)` gives row k's descriptor and
// its LDS index; the block's rows sit at LDS indices loc - rr .. loc - rr + w
// - 1.  Forward: y_B = inv(L_BB) y_B; backward: y_B = inv(L_BB)^T y_B and
// out[perm[j]] = scale y_j.  lpr lanes per row over the columns of the row of
// the inverse, eight loads a lane in flight (fixed-order sums); the results
// are staged in tmp / tloc (rows of one block read each other's inputs) and
// written back after all rows are done.
template <bool FWD, class RowOf>
__device__ inline void split_dense(const LdlDev &L, const SolveTask &t, int cnt, int lpr,
                                   RowOf row_of, double2 *ys, double2 *tmp, int *tloc) {
    const int grp = threadIdx.x / lpr, gl = threadIdx.x % lpr, ngrp = SPLIT_THREADS / lpr;
    const double2 *inv = (FWD ? L.invL : L.invLT) + (int64_t)t.factor * L.ndense;
    for (int k0 = 0; k0 < cnt; k0 += ngrp) {
        const int k = k0 + grp;
        double sx = 0.0, sy = 0.0;
        int loc = 0, perm = 0;
        if (k < cnt) {
            const LdlRow d = row_of(k, loc);
            perm = d.perm;
            const double2 *row = inv + d.doff + (int64_t)d.rr * d.w;
            const double2 *yb = ys + (loc - d.rr);
            const int c0 = FWD ? 0 : d.rr, c1 = FWD ? d.rr + 1 : d.w;
            for (int cb = c0 + gl; cb < c1; cb += 8 * lpr) {
                double2 v[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int c = cb + u * lpr;
                    v[u] = c < c1 ? row[c] : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int c = cb + u * lpr;
                    if (c < c1) {
                        const double2 p = cmul(v[u], yb[c]);
                        sx += p.x;
                        sy += p.y;
                    }
                }
            }
        }
        const double2 acc = group_sum(sx, sy, lpr);
        if (k < cnt && gl == 0) {
            tmp[k] = acc;
            tloc[k] = loc;
            if (!FWD) t.out[perm] = cmul(t.scale, acc);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < cnt; k += SPLIT_THREADS) ys[tloc[k]] = tmp[k];
    __syncthreads();
}

// Bottom subtree s = blockIdx.x of task blockIdx.y; LDS: the subtree's rows.
// Every row's own term (forward: in[perm[j]]; backward: D^{-1}_j times its
// forward result) is loaded for all rows at once, and with P.desc_lds the
// rows' descriptors are kept in LDS, so that a height costs one global round
// trip in each phase.  With P.top_levels the top rows are solved by the level
// kernels from the global work vector, so the forward pass forms no partial
// sums.
template <bool FWD>
__global__ __launch_bounds__(SPLIT_THREADS) void ldl_sub_kernel(LdlDev L, LdlSplitDev P,
                                                                TaskList tasks) {
    // sub_rows rows; hrows staged results and their indices; descriptors
    extern __shared__ double2 ys[];
    __shared__ int hp[LDL_SPLIT_MAX_H + 1];
    double2 *tmp = ys + P.sub_rows;
    int *tloc = reinterpret_cast<int *>(tmp + P.hrows);
    LdlRow *dl = reinterpret_cast<LdlRow *>(tmp + ldl_split_desc_off(P.hrows));
    const SolveTask t = task_of(tasks, blockIdx.y);
    const int s = blockIdx.x, r0 = P.sub_r0[s], r1 = P.sub_r1[s];
    const int grp = threadIdx.x >> 4, gl = threadIdx.x & 15, ngrp = SPLIT_THREADS / 16;
    double2 *z = t.work + L.n;
    if (threadIdx.x <= P.H) hp[threadIdx.x] = P.sub_hptr[s * P.H + threadIdx.x];
    __syncthreads();
    const int k0s = hp[0], nk = hp[P.H] - k0s;
    for (int k = threadIdx.x; k < nk; k += SPLIT_THREADS) {
        // (copied as three 16-byte words: {j, perm, s0, w}, ranges, dense)
        const int4 *src = reinterpret_cast<const int4 *>(P.sdesc + k0s + k);
        const int4 a = src[0], b = src[1], c = src[2];
        if (P.desc_lds) {
            int4 *dst = reinterpret_cast<int4 *>(dl + k);
            dst[0] = a;
            dst[1] = b;
            dst[2] = c;
        }
        const int j = a.x, perm = a.y;
        ys[j - r0] = FWD ? t.in[perm] : cmul(L.Dinv[(int64_t)t.factor * L.n + j], z[j]);
    }
    __syncthreads();
    // (an LDS pointer is never offset below its array: the row index is
    // taken relative to the subtree's first row instead)
    auto dsc = [&](int k) {
        const int4 *src = P.desc_lds ? reinterpret_cast<const int4 *>(dl + (k - k0s))
                                     : reinterpret_cast<const int4 *>(P.sdesc + k);
        const int4 a = src[0], b = src[1], c = src[2];
        return LdlRow{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
    };
    const double2 *val = (FWD ? L.Lcsr : L.Lcsc) + (int64_t)t.factor * L.nnz;
    for (int hi = 0; hi < P.H; hi++) {
        const int h = FWD ? hi : P.H - 1 - hi;
        const int a = hp[h], e = hp[h + 1];
        if (a == e) continue;   // uniform over the workgroup
        const int lpr = split_lanes(e - a);
        const int hg = threadIdx.x / lpr, hl = threadIdx.x % lpr, nhg = SPLIT_THREADS / lpr;
        for (int k0 = a; k0 < e; k0 += nhg) {
            const int k = k0 + hg;
            double sx = 0.0, sy = 0.0;
            int loc = 0;
            if (k < e) {
                const LdlRow d = dsc(k);
                loc = d.j - r0;
                // four entries a lane per round, all loads issued before the sums
                const int e0 = FWD ? d.fx : d.bx, e1 = FWD ? d.fy : d.by;
                for (int q0 = e0 + hl; q0 < e1; q0 += 4 * lpr) {
                    double2 v[4], x[4];
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const int q = q0 + lpr * u;
                        v[u] = make_double2(0.0, 0.0);
                        x[u] = make_double2(0.0, 0.0);
                        if (q < e1) {
                            v[u] = val[q];
                            if (FWD) {
                                x[u] = ys[L.Rj[q] - r0];
                            } else {
                                const int i = L.Li[q];
                                x[u] = q < d.bsplit ? ys[i - r0] : z[i];
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        if (q0 + lpr * u < e1) {
                            const double2 p = cmul(v[u], x[u]);
                            sx += p.x;
                            sy += p.y;
                        }
                    }
                }
            }
            const double2 acc = group_sum(sx, sy, lpr);
            if (k < e && hl == 0) ys[loc] = make_double2(ys[loc].x - acc.x, ys[loc].y - acc.y);
        }
        __syncthreads();
        split_dense<FWD>(L, t, e - a, lpr,
                         [&](int k, int &loc) {
                             const LdlRow d = dsc(a + k);
                             loc = d.j - r0;
                             return d;
                         },
                         ys, tmp, tloc);
    }
    if (!FWD) return;
    for (int r = threadIdx.x; r < r1 - r0; r += SPLIT_THREADS) z[r0 + r] = ys[r];
    if (P.top_levels) return;
    // partial sums of the top rows' external entries inside this subtree
    const double2 *vf = L.Lcsr + (int64_t)t.factor * L.nnz;
    double2 *part = t.work + 2 * L.n + (int64_t)s * P.ntop;
    for (int t0 = 0; t0 < P.ntop; t0 += ngrp) {
        const int tt = t0 + grp;
        double sx = 0.0, sy = 0.0;
        if (tt < P.ntop) {
            const int qb = P.part_b[(int64_t)s * P.ntop + tt], qe = P.part_e[(int64_t)s * P.ntop + tt];
            for (int q = qb + gl; q < qe; q += 16) {
                const double2 p = cmul(vf[q], ys[L.Rj[q] - r0]);
                sx += p.x;
                sy += p.y;
            }
        }
        const double2 acc = sum16(sx, sy);
        if (tt < P.ntop && gl == 0) part[tt] = acc;
    }
}

// Forward external update of a top row t: the subtrees' partial sums (in
// subtree order, lanes strided) plus its entries inside the top part; `yt`
// gives the value of top row u.
template <class YT>
__device__ inline double2 top_fwd_ext(const LdlDev &L, const LdlSplitDev &P, const SolveTask &t,
                                      int tt, int gl, YT yt) {
    double sx = 0.0, sy = 0.0;
    const double2 *part = t.work + 2 * L.n;
    for (int s = gl; s < P.nsub; s += 16) {
        const double2 v = part[(int64_t)s * P.ntop + tt];
        sx += v.x;
        sy += v.y;
    }
    const double2 *val = L.Lcsr + (int64_t)t.factor * L.nnz;
    for (int q = P.tf_ptr[tt] + gl; q < P.tf_ptr[tt + 1]; q += 16) {
        const double2 p = cmul(val[P.tf_pos[q]], yt(P.tf_col[q]));
        sx += p.x;
        sy += p.y;
    }
    return make_double2(sx, sy);
}

// The whole top part of task blockIdx.y in one workgroup; LDS: top rows.
__global__ __launch_bounds__(SPLIT_THREADS) void ldl_top_kernel(LdlDev L, LdlSplitDev P,
                                                                TaskList tasks) {
    extern __shared__ double2 ys[];   // ntop rows, then hrows staged results and indices
    double2 *tmp = ys + P.ntop;
    int *tloc = reinterpret_cast<int *>(tmp + P.hrows);
    const SolveTask t = task_of(tasks, blockIdx.y);
    const int grp = threadIdx.x >> 4, gl = threadIdx.x & 15, ngrp = SPLIT_THREADS / 16;
    auto yt = [&](int u) { return ys[u]; };
    for (int fb = 0; fb < 2; fb++) {
        const bool fwd = fb == 0;
        for (int hi = 0; hi < P.nht; hi++) {
            const int h = fwd ? hi : P.nht - 1 - hi;
            const int a = P.top_hptr[h], e = P.top_hptr[h + 1];
            if (a == e) continue;
            for (int k0 = a; k0 < e; k0 += ngrp) {
                const int k = k0 + grp;
                double2 acc = make_double2(0.0, 0.0);
                int tt = 0;
                if (k < e) {
                    tt = P.tlist[k];
                    if (fwd) {
                        acc = top_fwd_ext(L, P, t, tt, gl, yt);
                    } else {
                        const double2 *val = L.Lcsc + (int64_t)t.factor * L.nnz;
                        for (int q = P.tb_ptr[tt] + gl; q < P.tb_ptr[tt + 1]; q += 16) {
                            const double2 p = cmul(val[P.tb_pos[q]], ys[P.tb_row[q]]);
                            acc.x += p.x;
                            acc.y += p.y;
                        }
                    }
                }
                acc = sum16(acc.x, acc.y);
                if (k < e && gl == 0) {
                    const int j = P.top_row[tt];
                    const double2 base = fwd ? t.in[L.perm[j]]
                                             : cmul(L.Dinv[(int64_t)t.factor * L.n + j], ys[tt]);
                    ys[tt] = make_double2(base.x - acc.x, base.y - acc.y);
                }
            }
            __syncthreads();
            auto row_of = [&](int k, int &loc) {
                loc = P.tlist[a + k];
                return L.jrow[P.top_row[loc]];
            };
            if (fwd) split_dense<true>(L, t, e - a, 16, row_of, ys, tmp, tloc);
            else split_dense<false>(L, t, e - a, 16, row_of, ys, tmp, tloc);
        }
    }
    for (int u = threadIdx.x; u < P.ntop; u += SPLIT_THREADS) t.work[L.n + P.top_row[u]] = ys[u];
}

// Forward external update of the top rows of height H + h (level by level
// form of the top part): 16 lanes per row, grid (ceil(rows / 16), tasks).
__global__ __launch_bounds__(256) void ldl_top_ext_kernel(LdlDev L, LdlSplitDev P,
                                                          TaskList tasks, int h) {
    const SolveTask t = task_of(tasks, blockIdx.y);
    const int a = P.top_hptr[h], e = P.top_hptr[h + 1];
    const int k = a + blockIdx.x * 16 + (threadIdx.x >> 4), gl = threadIdx.x & 15;
    double2 acc = make_double2(0.0, 0.0);
    int tt = 0;
    if (k < e) {
        tt = P.tlist[k];
        acc = top_fwd_ext(L, P, t, tt, gl, [&](int u) { return t.work[L.n + P.top_row[u]]; });
    }
    acc = sum16(acc.x, acc.y);
    if (k < e && gl == 0) {
        const int j = P.top_row[tt];
        const double2 base = t.in[L.perm[j]];
        t.work[j] = make_double2(base.x - acc.x, base.y - acc.y);
    }
}

// out_r[i] = alpha (C0 u_r[i] - sum_j A_j s_{r,j}[i])
struct PadeArgs {
    PadeCoef pc;
    double2 alpha;
    const double2 *alpha_v, *u, *sv;
    int64_t ustride, sstride, vstride;
    double2 *out;
    int64_t ostride;
};
__device__ inline void pade_sum_row(int i, int64_t r, const PadeArgs &a) {
    const double2 *u = a.u + r * a.ustride, *sv = a.sv + r * a.vstride;
    double2 acc = cmul(a.pc.C0, u[i]);
    for (int j = 0; j < a.pc.np; j++) {
        const double2 p = cmul(a.pc.A[j], sv[j * a.sstride + i]);
        acc.x -= p.x;
        acc.y -= p.y;
    }
    a.out[r * a.ostride + i] = cmul(a.alpha_v ? a.alpha_v[i] : a.alpha, acc);
}

// out_b[i] = sum_e V_e in_b[col_e]  (real sparse matrix, complex vectors)
struct SpmvArgs {
    const int32_t *gptr, *gcol;
    const double *V;
    const double2 *in;
    int64_t istride;
    double2 *out;
    int64_t ostride;
};
__device__ inline void spmv_row(int i, int64_t b, const SpmvArgs &a) {
    const double2 *x = a.in + b * a.istride;
    double2 acc = make_double2(0.0, 0.0);
    for (int e = a.gptr[i]; e < a.gptr[i + 1]; e++) {
        const double2 v = x[a.gcol[e]];
        acc.x += a.V[e] * v.x;
        acc.y += a.V[e] * v.y;
    }
    a.out[b * a.ostride + i] = acc;
}

// Pade sums of right-hand side blockIdx.y (blockIdx.y < npade), then mass
// products of block blockIdx.y - npade, in one launch.
__global__ __launch_bounds__(256) void pade_spmv_kernel(int n, int npade, PadeArgs pa,
                                                        SpmvArgs ma) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int y = blockIdx.y;
    if (y < npade) pade_sum_row(i, y, pa);
    else spmv_row(i, y - npade, ma);
}

// Two Pade sums per right-hand side: by pa for blockIdx.y < nrhs, by pb for
// right-hand side blockIdx.y - nrhs.
__global__ __launch_bounds__(256) void pade_pair_kernel(int n, int nrhs, PadeArgs pa,
                                                        PadeArgs pb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int y = blockIdx.y;
    if (y < nrhs) pade_sum_row(i, y, pa);
    else pade_sum_row(i, y - nrhs, pb);
}

}   // namespace

int ldl_split_max_lds() {
    static const int lds = [] {
        int dev = 0, bytes = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess)
            bytes = 65536;
        return bytes;
    }();
    return lds;
}

size_t ldl_split_lds(int rows, int hrows, int desc_rows) {
    return (size_t)(rows + ldl_split_desc_off(hrows)) * sizeof(double2) +
           (size_t)desc_rows * sizeof(LdlRow);
}

int ldl_split_max_sub_rows() {
    return std::min(8192, ldl_split_max_lds() / (int)sizeof(double2));
}

void launch_ldl_solve(const LdlDev &L, const LdlSplitDev &P, TaskList tasks, int ntasks, int nrhs,
                      hipStream_t s) {
    Timer tm("osrc_ldl_solve", s);
    tasks.nbase = ntasks;
    const unsigned gy = (unsigned)(ntasks * nrhs);
    // Levels with many (small) blocks run in one launch per level; the top
    // levels, a few large separators with long rows, spread the external
    // update over one wavefront per row and then apply the dense inverses.
    const bool wide_lvl = nrhs < LVL_WIDE_MAX_RHS;
    auto level = [&](int l, bool fwd, auto fused, auto fused_wide, auto ext, auto ext_wide,
                     auto dense) {
        if (L.lbcount[l] >= LVL_FUSE_MIN_BLOCKS) {
            if (wide_lvl)
                hipLaunchKernelGGL(fused_wide, dim3(L.lbcount[l], gy), dim3(1024), 0, s, L, tasks,
                                   L.lbptr_h[l]);
            else
                hipLaunchKernelGGL(fused, dim3(L.lbcount[l], gy), dim3(256), 0, s, L, tasks,
                                   L.lbptr_h[l]);
        } else {
            const int rb = L.lptr_h[l], re = L.lptr_h[l + 1];
            if ((fwd ? L.lext_f : L.lext_b)[l] > LDL_WIDE_EXT * (int64_t)L.lrcount[l])
                hipLaunchKernelGGL(ext_wide, dim3(L.lrcount[l], gy), dim3(256), 0, s, L, tasks, rb,
                                   re);
            else
                hipLaunchKernelGGL(ext, dim3((L.lrcount[l] + 3) / 4, gy), dim3(256), 0, s, L, tasks,
                                   rb, re);
            hipLaunchKernelGGL(dense, dim3((L.lrcount[l] + 3) / 4, gy), dim3(256), 0, s, L, tasks, rb,
                               re);
        }
        BEM_LAUNCH_CHECK();
    };
    auto fwd_level = [&](int l) {
        level(l, true, ldl_level_kernel<true, 256>, ldl_level_kernel<true, 1024>,
              ldl_ext_kernel<true, false>,
              ldl_ext_kernel<true, true>, ldl_dense_kernel<true>);
    };
    auto bwd_level = [&](int l) {
        level(l, false, ldl_level_kernel<false, 256>, ldl_level_kernel<false, 1024>,
              ldl_ext_kernel<false, false>,
              ldl_ext_kernel<false, true>, ldl_dense_kernel<false>);
    };
    if (P.ok) {
        static std::once_flag lds_once;   // dynamic LDS beyond 64 KiB for the split kernels
        std::call_once(lds_once, [] {
            const int bytes = ldl_split_max_lds();
            (void)hipFuncSetAttribute((const void *)ldl_sub_kernel<true>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
            (void)hipFuncSetAttribute((const void *)ldl_sub_kernel<false>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
            (void)hipFuncSetAttribute((const void *)ldl_top_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
            (void)hipGetLastError();
        });
        const size_t sub_lds = ldl_split_lds(P.sub_rows, P.hrows, P.desc_lds ? P.sub_rows : 0);
        hipLaunchKernelGGL(ldl_sub_kernel<true>, dim3(P.nsub, gy), dim3(SPLIT_THREADS), sub_lds, s,
                           L, P, tasks);
        BEM_LAUNCH_CHECK();
        if (P.ntop > 0 && P.top_levels) {
            // top levels H .. nlev - 1 by the level kernels, forward then backward
            for (int l = P.H; l < L.nlev; l++) fwd_level(l);
            for (int l = L.nlev - 1; l >= P.H; l--) bwd_level(l);
        } else if (P.ntop > 0 && P.top_single) {
            hipLaunchKernelGGL(ldl_top_kernel, dim3(1, gy), dim3(SPLIT_THREADS),
                               ldl_split_lds(P.ntop, P.hrows, 0), s, L, P, tasks);
            BEM_LAUNCH_CHECK();
        } else if (P.ntop > 0) {
            // top levels H .. H + nht - 1 of the global schedule, forward then backward
            for (int h = 0; h < P.nht; h++) {
                const int lev = P.H + h, rb = L.lptr_h[lev], re = L.lptr_h[lev + 1];
                hipLaunchKernelGGL(ldl_top_ext_kernel, dim3((L.lrcount[lev] + 15) / 16, gy),
                                   dim3(256), 0, s, L, P, tasks, h);
                hipLaunchKernelGGL(ldl_dense_kernel<true>, dim3((L.lrcount[lev] + 3) / 4, gy),
                                   dim3(256), 0, s, L, tasks, rb, re);
                BEM_LAUNCH_CHECK();
            }
            for (int h = P.nht - 1; h >= 0; h--) {
                const int lev = P.H + h, rb = L.lptr_h[lev], re = L.lptr_h[lev + 1];
                hipLaunchKernelGGL((ldl_ext_kernel<false, false>),
                                   dim3((L.lrcount[lev] + 3) / 4, gy), dim3(256), 0, s, L, tasks,
                                   rb, re);
                hipLaunchKernelGGL(ldl_dense_kernel<false>, dim3((L.lrcount[lev] + 3) / 4, gy),
                                   dim3(256), 0, s, L, tasks, rb, re);
                BEM_LAUNCH_CHECK();
            }
        }
        hipLaunchKernelGGL(ldl_sub_kernel<false>, dim3(P.nsub, gy), dim3(SPLIT_THREADS), sub_lds,
                           s, L, P, tasks);
        BEM_LAUNCH_CHECK();
        return;
    }
    for (int l = 0; l < L.nlev; l++) fwd_level(l);
    for (int l = L.nlev - 1; l >= 0; l--) bwd_level(l);
}

void launch_pade_sum_spmv(int n, const PadeCoef &pc, double2 alpha, const double2 *alpha_v,
                          const double2 *u, int64_t ustride, const double2 *sv, int64_t sstride,
                          int64_t vstride, double2 *out, int64_t ostride, int npade,
                          const int32_t *gptr, const int32_t *gcol, const double *V,
                          const double2 *in, int64_t istride, double2 *mout, int64_t mstride,
                          int nspmv, hipStream_t s) {
    const PadeArgs pa{pc, alpha, alpha_v, u, sv, ustride, sstride, vstride, out, ostride};
    const SpmvArgs ma{gptr, gcol, V, in, istride, mout, mstride};
    hipLaunchKernelGGL(pade_spmv_kernel, dim3((n + 255) / 256, npade + nspmv), dim3(256), 0, s, n,
                       npade, pa, ma);
    BEM_LAUNCH_CHECK();
}

void launch_pade_pair(int n, const PadeCoef &pc, double2 alpha, const double2 *alpha_v,
                      const double2 *u, int64_t ustride, const double2 *sv, int64_t sstride,
                      int64_t vstride, double2 *out, int64_t ostride, const PadeCoef &pc2,
                      double2 alpha2, const double2 *alpha2_v, const double2 *u2,
                      const double2 *sv2, double2 *out2, int nrhs, hipStream_t s) {
    const PadeArgs pa{pc, alpha, alpha_v, u, sv, ustride, sstride, vstride, out, ostride};
    const PadeArgs pb{pc2, alpha2, alpha2_v, u2, sv2, ustride, sstride, vstride, out2, ostride};
    hipLaunchKernelGGL(pade_pair_kernel, dim3((n + 255) / 256, 2 * nrhs), dim3(256), 0, s, n,
                       nrhs, pa, pb);
    BEM_LAUNCH_CHECK();
}

void launch_pade_sum(int n, const PadeCoef &pc, double2 alpha, const double2 *alpha_v,
                     const double2 *u, int64_t ustride, const double2 *sv, int64_t sstride,
                     int64_t vstride, double2 *out, int64_t ostride, int nrhs, hipStream_t s) {
    launch_pade_sum_spmv(n, pc, alpha, alpha_v, u, ustride, sv, sstride, vstride, out, ostride,
                         nrhs, nullptr, nullptr, nullptr, nullptr, 0, nullptr, 0, 0, s);
}

void launch_spmv_real(int n, int nblk, const int32_t *gptr, const int32_t *gcol,
                      const double *V, const double2 *in, int64_t istride, double2 *out,
                      int64_t ostride, hipStream_t s) {
    launch_pade_sum_spmv(n, PadeCoef{}, make_double2(0.0, 0.0), nullptr, nullptr, 0, nullptr, 0,
                         0, nullptr, 0, 0, gptr, gcol, V, in, istride, out, ostride, nblk, s);
}

}   // namespace bem

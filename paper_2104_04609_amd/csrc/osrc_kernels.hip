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

constexpr int LVL_THREADS = 256;
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
// butterfly), grid (ceil(rows / 4), tasks).
template <bool FWD>
__global__ __launch_bounds__(256) void ldl_ext_kernel(LdlDev L, TaskList tasks, int lev) {
    const SolveTask t = task_of(tasks, blockIdx.y);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = L.lptr[lev] + blockIdx.x * 4 + wave;
    if (r >= L.lptr[lev + 1]) return;
    const int j = L.lrow[r];
    double2 *y = t.work, *z = t.work + L.n;
    const double2 *val = (FWD ? L.Lcsr : L.Lcsc) + (int64_t)t.factor * L.nnz;
    const int32_t *idx = FWD ? L.Rj : L.Li;
    const int2 rg = (FWD ? L.frange : L.brange)[j];
    double sx = 0.0, sy = 0.0;
#pragma unroll 4
    for (int e = rg.x + lane; e < rg.y; e += 64) {
        const double2 p = cmul(val[e], z[idx[e]]);
        sx += p.x;
        sy += p.y;
    }
    const double2 acc = lane_sum<64>(sx, sy);
    if (lane == 0) {
        const double2 base =
            FWD ? t.in[L.perm[j]] : cmul(L.Dinv[(int64_t)t.factor * L.n + j], z[j]);
        y[j] = make_double2(base.x - acc.x, base.y - acc.y);
    }
}

// Dense block products of a level: one wavefront per row (any block width),
// grid (ceil(rows / 4), tasks); y_B is complete (previous launch).
template <bool FWD>
__global__ __launch_bounds__(256) void ldl_dense_kernel(LdlDev L, TaskList tasks, int lev) {
    const SolveTask t = task_of(tasks, blockIdx.y);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = L.lptr[lev] + blockIdx.x * 4 + wave;
    if (r >= L.lptr[lev + 1]) return;
    const int j = L.lrow[r];
    const int b = L.blk[j], s0 = L.bstart[b], w = L.bstart[b + 1] - s0, rr = j - s0;
    const double2 *y = t.work;
    double2 *z = t.work + L.n;
    const double2 *row = (FWD ? L.invL : L.invLT) + (int64_t)t.factor * L.ndense + L.doff[b] +
                         (int64_t)rr * w;
    const double2 p = dense_row<FWD, 64>(row, rr, w, lane, [&](int c) { return y[s0 + c]; });
    const double2 acc = lane_sum<64>(p.x, p.y);
    if (lane == 0) {
        z[j] = acc;
        if (!FWD) t.out[L.perm[j]] = cmul(t.scale, acc);
    }
}

// One level of the sweep (levels of many small blocks): workgroup (block,
// task) forms the external updates of its rows (16 lanes per row, fixed
// butterfly; rows of finished levels only) into LDS, then the dense block
// product (16 lanes per row).
template <bool FWD>
__global__ __launch_bounds__(LVL_THREADS) void ldl_level_kernel(LdlDev L, TaskList tasks,
                                                                int lev) {
    __shared__ double2 tb[LDL_MAX_BLOCK];
    const SolveTask t = task_of(tasks, blockIdx.y);
    const int b = L.lblk[L.lbptr[lev] + blockIdx.x];
    const int s0 = L.bstart[b], w = L.bstart[b + 1] - s0;
    double2 *z = t.work + L.n;
    const double2 *val = (FWD ? L.Lcsr : L.Lcsc) + (int64_t)t.factor * L.nnz;
    const int32_t *idx = FWD ? L.Rj : L.Li;
    const int grp = threadIdx.x >> 4, gl = threadIdx.x & 15;
    for (int r0 = 0; r0 < w; r0 += LVL_THREADS / 16) {
        const int r = r0 + grp;
        double sx = 0.0, sy = 0.0;
        if (r < w) {
            const int2 rg = (FWD ? L.frange : L.brange)[s0 + r];
#pragma unroll 4
            for (int e = rg.x + gl; e < rg.y; e += 16) {
                const double2 p = cmul(val[e], z[idx[e]]);
                sx += p.x;
                sy += p.y;
            }
        }
        const double2 acc = lane_sum<16>(sx, sy);
        if (r < w && gl == 0) {
            const int j = s0 + r;
            const double2 base =
                FWD ? t.in[L.perm[j]] : cmul(L.Dinv[(int64_t)t.factor * L.n + j], z[j]);
            tb[r] = make_double2(base.x - acc.x, base.y - acc.y);
        }
    }
    __syncthreads();
    const double2 *dense = (FWD ? L.invL : L.invLT) + (int64_t)t.factor * L.ndense + L.doff[b];
    for (int r0 = 0; r0 < w; r0 += LVL_THREADS / 16) {
        const int r = r0 + grp;
        double2 p = make_double2(0.0, 0.0);
        if (r < w) p = dense_row<FWD, 16>(dense + (int64_t)r * w, r, w, gl, [&](int c) { return tb[c]; });
        const double2 acc = lane_sum<16>(p.x, p.y);
        if (r < w && gl == 0) {
            z[s0 + r] = acc;
            if (!FWD) t.out[L.perm[s0 + r]] = cmul(t.scale, acc);
        }
    }
}

// ------------------------------------------------ two-part (split) solve
// Bottom subtrees: one workgroup per (subtree, task) holds the subtree's rows
// in LDS (row j at j - r0) and runs its heights in order (forward) or in
// reverse (backward), an external update phase (16 lanes per row, fixed
// butterfly) then a dense phase (one thread per row, at most SPLIT_ROWS_PER
// _THREAD rows per thread kept in registers until the whole height is done).
// The forward kernel also forms, for every top row, the partial sum of its
// external entries inside the subtree.  The top part: one workgroup per task
// (forward, D^{-1}, backward) with its rows in LDS at their local index, or
// level by level through the global work vector.
constexpr int SPLIT_THREADS = 1024;
constexpr int SPLIT_ROWS_PER_THREAD = 4;

// Sum of 16 lanes (fixed butterfly; all 16 lanes of the group take part).
__device__ inline double2 sum16(double sx, double sy) {
    for (int o = 8; o > 0; o >>= 1) {
        sx += __shfl_xor(sx, o, 16);
        sy += __shfl_xor(sy, o, 16);
    }
    return make_double2(sx, sy);
}

// Dense phase on `cnt` rows: rows[k] -> (global row j, LDS index loc) by
// `row_of`; the block's rows sit at LDS indices loc - rr .. loc - rr + w - 1.
// Forward: y_B = inv(L_BB) y_B; backward: y_B = inv(L_BB)^T y_B and
// out[perm[j]] = scale y_j.
template <bool FWD, class RowOf>
__device__ inline void split_dense(const LdlDev &L, const SolveTask &t, int cnt, RowOf row_of,
                                   double2 *ys) {
    double2 res[SPLIT_ROWS_PER_THREAD];
    for (int i = 0; i < SPLIT_ROWS_PER_THREAD; i++) {
        const int k = threadIdx.x + i * SPLIT_THREADS;
        if (k >= cnt) break;
        int j, loc;
        row_of(k, j, loc);
        const int b = L.blk[j], s0 = L.bstart[b], w = L.bstart[b + 1] - s0, rr = j - s0;
        const double2 *dense = (FWD ? L.invLT : L.invL) + (int64_t)t.factor * L.ndense + L.doff[b];
        const double2 *yb = ys + (loc - rr);
        double2 a[4];
        for (int q = 0; q < 4; q++) a[q] = make_double2(0.0, 0.0);
        const int c0 = FWD ? 0 : rr, c1 = FWD ? rr + 1 : w;
        int c = c0;
        for (; c + 4 <= c1; c += 4) {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const double2 p = cmul(dense[(int64_t)(c + q) * w + rr], yb[c + q]);
                a[q].x += p.x;
                a[q].y += p.y;
            }
        }
        for (; c < c1; c++) {
            const double2 p = cmul(dense[(int64_t)c * w + rr], yb[c]);
            a[0].x += p.x;
            a[0].y += p.y;
        }
        res[i] = make_double2((a[0].x + a[1].x) + (a[2].x + a[3].x),
                              (a[0].y + a[1].y) + (a[2].y + a[3].y));
    }
    __syncthreads();
    for (int i = 0; i < SPLIT_ROWS_PER_THREAD; i++) {
        const int k = threadIdx.x + i * SPLIT_THREADS;
        if (k >= cnt) break;
        int j, loc;
        row_of(k, j, loc);
        ys[loc] = res[i];
        if (!FWD) t.out[L.perm[j]] = cmul(t.scale, res[i]);
    }
    __syncthreads();
}

// Bottom subtree s = blockIdx.x of task blockIdx.y; LDS: the subtree's rows.
template <bool FWD>
__global__ __launch_bounds__(SPLIT_THREADS) void ldl_sub_kernel(LdlDev L, LdlSplitDev P,
                                                                TaskList tasks) {
    extern __shared__ double2 ys[];
    const SolveTask t = task_of(tasks, blockIdx.y);
    const int s = blockIdx.x, r0 = P.sub_r0[s], r1 = P.sub_r1[s];
    const int grp = threadIdx.x >> 4, gl = threadIdx.x & 15, ngrp = SPLIT_THREADS / 16;
    double2 *z = t.work + L.n;
    if (!FWD) {
        for (int r = threadIdx.x; r < r1 - r0; r += SPLIT_THREADS) ys[r] = z[r0 + r];
        __syncthreads();
    }
    for (int hi = 0; hi < P.H; hi++) {
        const int h = FWD ? hi : P.H - 1 - hi;
        const int a = P.sub_hptr[s * P.H + h], e = P.sub_hptr[s * P.H + h + 1];
        if (a == e) continue;   // uniform over the workgroup
        for (int k0 = a; k0 < e; k0 += ngrp) {
            const int k = k0 + grp;
            double sx = 0.0, sy = 0.0;
            int j = 0;
            if (k < e) {
                j = P.srow[k];
                if (FWD) {
                    const double2 *val = L.Lcsr + (int64_t)t.factor * L.nnz;
                    const int2 rg = L.frange[j];
                    for (int q = rg.x + gl; q < rg.y; q += 16) {
                        const double2 p = cmul(val[q], ys[L.Rj[q] - r0]);
                        sx += p.x;
                        sy += p.y;
                    }
                } else {
                    const double2 *val = L.Lcsc + (int64_t)t.factor * L.nnz;
                    const int2 rg = L.brange[j];
                    const int split = P.bsplit[j];
                    for (int q = rg.x + gl; q < rg.y; q += 16) {
                        const int i = L.Li[q];
                        const double2 p = cmul(val[q], q < split ? ys[i - r0] : z[i]);
                        sx += p.x;
                        sy += p.y;
                    }
                }
            }
            const double2 acc = sum16(sx, sy);
            if (k < e && gl == 0) {
                const double2 base = FWD ? t.in[L.perm[j]]
                                         : cmul(L.Dinv[(int64_t)t.factor * L.n + j], ys[j - r0]);
                ys[j - r0] = make_double2(base.x - acc.x, base.y - acc.y);
            }
        }
        __syncthreads();
        split_dense<FWD>(L, t, e - a,
                         [&](int k, int &j, int &loc) {
                             j = P.srow[a + k];
                             loc = j - r0;
                         },
                         ys);
    }
    if (!FWD) return;
    for (int r = threadIdx.x; r < r1 - r0; r += SPLIT_THREADS) z[r0 + r] = ys[r];
    // partial sums of the top rows' external entries inside this subtree
    const double2 *val = L.Lcsr + (int64_t)t.factor * L.nnz;
    double2 *part = t.work + 2 * L.n + (int64_t)s * P.ntop;
    for (int t0 = 0; t0 < P.ntop; t0 += ngrp) {
        const int tt = t0 + grp;
        double sx = 0.0, sy = 0.0;
        if (tt < P.ntop) {
            const int qb = P.part_b[(int64_t)s * P.ntop + tt], qe = P.part_e[(int64_t)s * P.ntop + tt];
            for (int q = qb + gl; q < qe; q += 16) {
                const double2 p = cmul(val[q], ys[L.Rj[q] - r0]);
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
    extern __shared__ double2 ys[];
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
            auto row_of = [&](int k, int &j, int &loc) {
                loc = P.tlist[a + k];
                j = P.top_row[loc];
            };
            if (fwd) split_dense<true>(L, t, e - a, row_of, ys);
            else split_dense<false>(L, t, e - a, row_of, ys);
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

// out_r[i] = alpha (C0 u_r[i] - sum_j A_j s_{r,j}[i]), r = blockIdx.y
__global__ __launch_bounds__(256) void pade_sum_kernel(int n, PadeCoef pc, double2 alpha,
                                                       const double2 *__restrict__ alpha_v,
                                                       const double2 *__restrict__ u,
                                                       int64_t ustride,
                                                       const double2 *__restrict__ sv,
                                                       int64_t sstride, int64_t vstride,
                                                       double2 *__restrict__ out,
                                                       int64_t ostride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t r = blockIdx.y;
    u += r * ustride;
    sv += r * vstride;
    out += r * ostride;
    double2 acc = cmul(pc.C0, u[i]);
    for (int j = 0; j < pc.np; j++) {
        const double2 p = cmul(pc.A[j], sv[j * sstride + i]);
        acc.x -= p.x;
        acc.y -= p.y;
    }
    out[i] = cmul(alpha_v ? alpha_v[i] : alpha, acc);
}

// out_b[i] = sum_e V_e in_b[col_e]  (real sparse matrix, complex vectors),
// block b = blockIdx.y
__global__ __launch_bounds__(256) void spmv_real_kernel(int n, const int32_t *__restrict__ gptr,
                                                        const int32_t *__restrict__ gcol,
                                                        const double *__restrict__ V,
                                                        const double2 *__restrict__ in,
                                                        int64_t istride,
                                                        double2 *__restrict__ out,
                                                        int64_t ostride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 *x = in + (int64_t)blockIdx.y * istride;
    double2 acc = make_double2(0.0, 0.0);
    for (int e = gptr[i]; e < gptr[i + 1]; e++) {
        const double2 v = x[gcol[e]];
        acc.x += V[e] * v.x;
        acc.y += V[e] * v.y;
    }
    out[(int64_t)blockIdx.y * ostride + i] = acc;
}

}   // namespace

int ldl_split_max_sub_rows() {
    static const int rows = [] {
        int dev = 0, bytes = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess)
            bytes = 65536;
        return std::min(8192, bytes / (int)sizeof(double2));
    }();
    return rows;
}

void launch_ldl_solve(const LdlDev &L, const LdlSplitDev &P, TaskList tasks, int ntasks, int nrhs,
                      hipStream_t s) {
    Timer tm("osrc_ldl_solve", s);
    tasks.nbase = ntasks;
    const unsigned gy = (unsigned)(ntasks * nrhs);
    if (P.ok) {
        static std::once_flag lds_once;   // dynamic LDS beyond 64 KiB for the split kernels
        std::call_once(lds_once, [] {
            const int bytes = ldl_split_max_sub_rows() * (int)sizeof(double2);
            (void)hipFuncSetAttribute((const void *)ldl_sub_kernel<true>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
            (void)hipFuncSetAttribute((const void *)ldl_sub_kernel<false>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
            (void)hipFuncSetAttribute((const void *)ldl_top_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
            (void)hipGetLastError();
        });
        const size_t sub_lds = (size_t)P.sub_rows * sizeof(double2);
        hipLaunchKernelGGL(ldl_sub_kernel<true>, dim3(P.nsub, gy), dim3(SPLIT_THREADS), sub_lds, s,
                           L, P, tasks);
        BEM_LAUNCH_CHECK();
        if (P.ntop > 0 && P.top_single) {
            hipLaunchKernelGGL(ldl_top_kernel, dim3(1, gy), dim3(SPLIT_THREADS),
                               (size_t)P.ntop * sizeof(double2), s, L, P, tasks);
            BEM_LAUNCH_CHECK();
        } else if (P.ntop > 0) {
            // top levels H .. H + nht - 1 of the global schedule, forward then backward
            for (int h = 0; h < P.nht; h++) {
                const int lev = P.H + h;
                hipLaunchKernelGGL(ldl_top_ext_kernel, dim3((L.lrcount[lev] + 15) / 16, gy),
                                   dim3(256), 0, s, L, P, tasks, h);
                hipLaunchKernelGGL(ldl_dense_kernel<true>, dim3((L.lrcount[lev] + 3) / 4, gy),
                                   dim3(256), 0, s, L, tasks, lev);
                BEM_LAUNCH_CHECK();
            }
            for (int h = P.nht - 1; h >= 0; h--) {
                const int lev = P.H + h;
                hipLaunchKernelGGL(ldl_ext_kernel<false>, dim3((L.lrcount[lev] + 3) / 4, gy),
                                   dim3(256), 0, s, L, tasks, lev);
                hipLaunchKernelGGL(ldl_dense_kernel<false>, dim3((L.lrcount[lev] + 3) / 4, gy),
                                   dim3(256), 0, s, L, tasks, lev);
                BEM_LAUNCH_CHECK();
            }
        }
        hipLaunchKernelGGL(ldl_sub_kernel<false>, dim3(P.nsub, gy), dim3(SPLIT_THREADS), sub_lds,
                           s, L, P, tasks);
        BEM_LAUNCH_CHECK();
        return;
    }
    // Levels with many (small) blocks run in one launch per level; the top
    // levels, a few large separators with long rows, spread the external
    // update over one wavefront per row and then apply the dense inverses.
    auto level = [&](int l, auto fused, auto ext, auto dense) {
        if (L.lbcount[l] >= LVL_FUSE_MIN_BLOCKS) {
            hipLaunchKernelGGL(fused, dim3(L.lbcount[l], gy), dim3(LVL_THREADS), 0, s, L, tasks, l);
        } else {
            hipLaunchKernelGGL(ext, dim3((L.lrcount[l] + 3) / 4, gy), dim3(256), 0, s, L, tasks, l);
            hipLaunchKernelGGL(dense, dim3((L.lrcount[l] + 3) / 4, gy), dim3(256), 0, s, L, tasks, l);
        }
        BEM_LAUNCH_CHECK();
    };
    for (int l = 0; l < L.nlev; l++)
        level(l, ldl_level_kernel<true>, ldl_ext_kernel<true>, ldl_dense_kernel<true>);
    for (int l = L.nlev - 1; l >= 0; l--)
        level(l, ldl_level_kernel<false>, ldl_ext_kernel<false>, ldl_dense_kernel<false>);
}

void launch_pade_sum(int n, const PadeCoef &pc, double2 alpha, const double2 *alpha_v,
                     const double2 *u, int64_t ustride, const double2 *sv, int64_t sstride,
                     int64_t vstride, double2 *out, int64_t ostride, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(pade_sum_kernel, dim3((n + 255) / 256, nrhs), dim3(256), 0, s, n, pc,
                       alpha, alpha_v, u, ustride, sv, sstride, vstride, out, ostride);
    BEM_LAUNCH_CHECK();
}

void launch_spmv_real(int n, int nblk, const int32_t *gptr, const int32_t *gcol,
                      const double *V, const double2 *in, int64_t istride, double2 *out,
                      int64_t ostride, hipStream_t s) {
    hipLaunchKernelGGL(spmv_real_kernel, dim3((n + 255) / 256, nblk), dim3(256), 0, s, n, gptr,
                       gcol, V, in, istride, out, ostride);
    BEM_LAUNCH_CHECK();
}

}   // namespace bem

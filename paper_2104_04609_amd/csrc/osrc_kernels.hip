// Device kernels of the OSRC preconditioner: batched block-LDL^T solves over
// the nested-dissection tree (all shifted systems share one pattern) and the
// elementwise Pade partial-fraction sums.
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
// launches have finished.
//
// forward, block B = rows [s0, s0 + w):
//   y_j = in[perm[j]] - sum_{k < s0} L_jk y_k         (external update)
//   y_B = inv(L_BB) y_B                               (dense block inverse)
// backward (levels from the top down):
//   y_j = Dinv_j y_j - sum_{i >= s0 + w} L_ij y_i      (external update)
//   y_B = inv(L_BB)^T y_B;  out[perm[j]] = scale y_j
__device__ inline SolveTask task_of(const TaskList &tasks, int y) {
    const int b = y % tasks.nbase, r = y / tasks.nbase;
    SolveTask t = tasks.t[b];
    t.in += r * tasks.in_stride;
    t.out += r * tasks.out_stride;
    t.work += r * tasks.work_stride;
    return t;
}

// External update: one wavefront per row of the level (fixed-order
// butterfly reduction), grid (ceil(rows / 4), tasks).  In place: a row only
// reads rows of other (finished) blocks.
template <bool FWD>
__global__ __launch_bounds__(256) void ldl_ext_kernel(LdlDev L, TaskList tasks, int lev) {
    const SolveTask t = task_of(tasks, blockIdx.y);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = L.lptr[lev] + blockIdx.x * 4 + wave;
    if (r >= L.lptr[lev + 1]) return;
    const int j = L.lrow[r];
    double2 *y = t.work;
    const double2 *val = (FWD ? L.Lcsr : L.Lcsc) + (int64_t)t.factor * L.nnz;
    const int32_t *idx = FWD ? L.Rj : L.Li;
    const int2 rg = (FWD ? L.frange : L.brange)[j];
    double sx = 0.0, sy = 0.0;
    for (int e = rg.x + lane; e < rg.y; e += 64) {
        const double2 p = cmul(val[e], y[idx[e]]);
        sx += p.x;
        sy += p.y;
    }
    for (int o = 32; o > 0; o >>= 1) {
        sx += __shfl_xor(sx, o, 64);
        sy += __shfl_xor(sy, o, 64);
    }
    if (lane == 0) {
        const double2 base =
            FWD ? t.in[L.perm[j]] : cmul(L.Dinv[(int64_t)t.factor * L.n + j], y[j]);
        y[j] = make_double2(base.x - sx, base.y - sy);
    }
}

// Dense block inverse: workgroup (block, task).  Consecutive threads (rows)
// read consecutive addresses: invLT[c][r] forward, invL[c][r] backward.
template <bool FWD>
__global__ __launch_bounds__(LVL_THREADS) void ldl_dense_kernel(LdlDev L, TaskList tasks,
                                                                int lev) {
    __shared__ double2 tb[LDL_MAX_BLOCK];
    const SolveTask t = task_of(tasks, blockIdx.y);
    const int b = L.lblk[L.lbptr[lev] + blockIdx.x];
    const int s0 = L.bstart[b], w = L.bstart[b + 1] - s0;
    double2 *y = t.work;
    const double2 *dense = (FWD ? L.invLT : L.invL) + (int64_t)t.factor * L.ndense + L.doff[b];
    for (int r = threadIdx.x; r < w; r += LVL_THREADS) tb[r] = y[s0 + r];
    __syncthreads();
    for (int r = threadIdx.x; r < w; r += LVL_THREADS) {
        // eight independent partial sums (loads in flight), added in a fixed order
        double2 a[8];
        for (int k = 0; k < 8; k++) a[k] = make_double2(0.0, 0.0);
        const int c0 = FWD ? 0 : r, c1 = FWD ? r + 1 : w;
        int c = c0;
        for (; c + 8 <= c1; c += 8) {
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const double2 p = cmul(dense[(int64_t)(c + k) * w + r], tb[c + k]);
                a[k].x += p.x;
                a[k].y += p.y;
            }
        }
        for (; c < c1; c++) {
            const double2 p = cmul(dense[(int64_t)c * w + r], tb[c]);
            a[0].x += p.x;
            a[0].y += p.y;
        }
        double2 acc;
        acc.x = ((a[0].x + a[1].x) + (a[2].x + a[3].x)) + ((a[4].x + a[5].x) + (a[6].x + a[7].x));
        acc.y = ((a[0].y + a[1].y) + (a[2].y + a[3].y)) + ((a[4].y + a[5].y) + (a[6].y + a[7].y));
        y[s0 + r] = acc;
        if (!FWD) t.out[L.perm[s0 + r]] = cmul(t.scale, acc);
    }
}

// One level of the sweep: workgroup (block, task) first forms the external
// updates of its block's rows (16 lanes per row, fixed butterfly; rows of
// finished levels only) into LDS, then applies the dense block inverse.
// Consecutive threads (rows) read consecutive addresses of the inverse:
// invLT[c][r] forward, invL[c][r] backward.
template <bool FWD>
__global__ __launch_bounds__(LVL_THREADS) void ldl_level_kernel(LdlDev L, TaskList tasks,
                                                                int lev) {
    __shared__ double2 tb[LDL_MAX_BLOCK];
    const SolveTask t = task_of(tasks, blockIdx.y);
    const int b = L.lblk[L.lbptr[lev] + blockIdx.x];
    const int s0 = L.bstart[b], w = L.bstart[b + 1] - s0;
    double2 *y = t.work;
    const double2 *val = (FWD ? L.Lcsr : L.Lcsc) + (int64_t)t.factor * L.nnz;
    const int32_t *idx = FWD ? L.Rj : L.Li;
    const int grp = threadIdx.x >> 4, gl = threadIdx.x & 15;
    for (int r0 = 0; r0 < w; r0 += LVL_THREADS / 16) {
        const int r = r0 + grp;
        double sx = 0.0, sy = 0.0;
        if (r < w) {
            const int2 rg = (FWD ? L.frange : L.brange)[s0 + r];
            for (int e = rg.x + gl; e < rg.y; e += 16) {
                const double2 p = cmul(val[e], y[idx[e]]);
                sx += p.x;
                sy += p.y;
            }
        }
        for (int o = 8; o > 0; o >>= 1) {
            sx += __shfl_xor(sx, o, 16);
            sy += __shfl_xor(sy, o, 16);
        }
        if (r < w && gl == 0) {
            const int j = s0 + r;
            const double2 base =
                FWD ? t.in[L.perm[j]] : cmul(L.Dinv[(int64_t)t.factor * L.n + j], y[j]);
            tb[r] = make_double2(base.x - sx, base.y - sy);
        }
    }
    __syncthreads();
    const double2 *dense = (FWD ? L.invLT : L.invL) + (int64_t)t.factor * L.ndense + L.doff[b];
    for (int r = threadIdx.x; r < w; r += LVL_THREADS) {
        // eight independent partial sums (loads in flight), added in a fixed order
        double2 a[8];
        for (int k = 0; k < 8; k++) a[k] = make_double2(0.0, 0.0);
        const int c0 = FWD ? 0 : r, c1 = FWD ? r + 1 : w;
        int c = c0;
        for (; c + 8 <= c1; c += 8) {
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const double2 p = cmul(dense[(int64_t)(c + k) * w + r], tb[c + k]);
                a[k].x += p.x;
                a[k].y += p.y;
            }
        }
        for (; c < c1; c++) {
            const double2 p = cmul(dense[(int64_t)c * w + r], tb[c]);
            a[0].x += p.x;
            a[0].y += p.y;
        }
        double2 acc;
        acc.x = ((a[0].x + a[1].x) + (a[2].x + a[3].x)) + ((a[4].x + a[5].x) + (a[6].x + a[7].x));
        acc.y = ((a[0].y + a[1].y) + (a[2].y + a[3].y)) + ((a[4].y + a[5].y) + (a[6].y + a[7].y));
        y[s0 + r] = acc;
        if (!FWD) t.out[L.perm[s0 + r]] = cmul(t.scale, acc);
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

void launch_ldl_solve(const LdlDev &L, TaskList tasks, int ntasks, int nrhs, hipStream_t s) {
    Timer tm("osrc_ldl_solve", s);
    tasks.nbase = ntasks;
    const unsigned gy = (unsigned)(ntasks * nrhs);
    // Levels with many (small) blocks run in one launch per level; the top
    // levels, a few large separators with long rows, spread the external
    // update over one wavefront per row and then apply the dense inverses.
    auto level = [&](int l, auto fused, auto ext, auto dense) {
        if (L.lbcount[l] >= LVL_FUSE_MIN_BLOCKS) {
            hipLaunchKernelGGL(fused, dim3(L.lbcount[l], gy), dim3(LVL_THREADS), 0, s, L, tasks, l);
        } else {
            hipLaunchKernelGGL(ext, dim3((L.lrcount[l] + 3) / 4, gy), dim3(256), 0, s, L, tasks, l);
            hipLaunchKernelGGL(dense, dim3(L.lbcount[l], gy), dim3(LVL_THREADS), 0, s, L, tasks, l);
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

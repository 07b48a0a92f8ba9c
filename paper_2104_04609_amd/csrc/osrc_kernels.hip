// Device kernels of the OSRC preconditioner: batched level-scheduled sparse
// LDL^T solves (one workgroup per shifted system and right-hand side, all
// systems sharing one pattern) and the Pade combinations with the P1
// stiffness matrix.
#include "osrc_internal.h"

namespace bem {

namespace {

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

constexpr int LDL_THREADS = 1024;

// y[j] -= sum_e val[e] * y[idx[e]] for every row j of one level.  Wide levels:
// one thread per row; narrow levels (long separator rows): one wavefront per
// row with a fixed-order butterfly reduction.
__device__ inline void sweep_level(double2 *__restrict__ y, const int32_t *__restrict__ rows,
                                   int beg, int end, const int32_t *__restrict__ ptr,
                                   const int32_t *__restrict__ idx,
                                   const double2 *__restrict__ val) {
    const int tid = threadIdx.x;
    if (end - beg >= 64) {
        for (int r = beg + tid; r < end; r += LDL_THREADS) {
            const int j = rows[r];
            double2 acc = y[j];
            for (int e = ptr[j]; e < ptr[j + 1]; e++) {
                const double2 p = cmul(val[e], y[idx[e]]);
                acc.x -= p.x;
                acc.y -= p.y;
            }
            y[j] = acc;
        }
    } else {
        const int wave = tid >> 6, lane = tid & 63;
        for (int r = beg + wave; r < end; r += LDL_THREADS / 64) {
            const int j = rows[r];
            double sx = 0.0, sy = 0.0;
            for (int e = ptr[j] + lane; e < ptr[j + 1]; e += 64) {
                const double2 p = cmul(val[e], y[idx[e]]);
                sx += p.x;
                sy += p.y;
            }
            for (int o = 32; o > 0; o >>= 1) {
                sx += __shfl_xor(sx, o, 64);
                sy += __shfl_xor(sy, o, 64);
            }
            if (lane == 0) {
                double2 v = y[j];
                y[j] = make_double2(v.x - sx, v.y - sy);
            }
        }
    }
}

__global__ __launch_bounds__(LDL_THREADS) void ldl_solve_kernel(LdlDev L, TaskList tasks) {
    const SolveTask t = tasks.t[blockIdx.x];
    const int n = L.n;
    const double2 *Dinv = L.Dinv + (int64_t)t.factor * n;
    const double2 *Lr = L.Lcsr + (int64_t)t.factor * L.nnz;
    const double2 *Lc = L.Lcsc + (int64_t)t.factor * L.nnz;
    double2 *y = t.work;
    for (int i = threadIdx.x; i < n; i += LDL_THREADS) y[i] = t.in[L.perm[i]];
    __syncthreads();
    for (int l = 0; l < L.nfl; l++) {
        sweep_level(y, L.frow, L.fptr[l], L.fptr[l + 1], L.Rp, L.Rj, Lr);
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += LDL_THREADS) y[i] = cmul(y[i], Dinv[i]);
    __syncthreads();
    for (int l = 0; l < L.nbl; l++) {
        sweep_level(y, L.brow, L.bptr[l], L.bptr[l + 1], L.Lp, L.Li, Lc);
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += LDL_THREADS) t.out[L.perm[i]] = cmul(t.scale, y[i]);
}

// out[i] = C0 in[i] - c_i sum_e S_ie sum_j A_j s_j[col_e]
__global__ __launch_bounds__(256) void pade_combine_kernel(
    int n, const int32_t *__restrict__ gptr, const int32_t *__restrict__ gcol,
    const double *__restrict__ Sv, const double2 *__restrict__ cvert, PadeCoef pc,
    const double2 *__restrict__ in, const double2 *__restrict__ sv, int64_t sstride,
    double2 *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 acc = make_double2(0.0, 0.0);
    for (int e = gptr[i]; e < gptr[i + 1]; e++) {
        const int c = gcol[e];
        double2 t = make_double2(0.0, 0.0);
        for (int j = 0; j < pc.np; j++) {
            const double2 p = cmul(pc.A[j], sv[j * sstride + c]);
            t.x += p.x;
            t.y += p.y;
        }
        acc.x += Sv[e] * t.x;
        acc.y += Sv[e] * t.y;
    }
    const double2 w = cmul(cvert[i], acc);
    const double2 a = cmul(pc.C0, in[i]);
    out[i] = make_double2(a.x - w.x, a.y - w.y);
}

// out[i] = sum_e V_e in[col_e]  (real sparse matrix, complex vector), for
// nblk consecutive blocks of length n
__global__ __launch_bounds__(256) void spmv_real_kernel(int n, int nblk,
                                                        const int32_t *__restrict__ gptr,
                                                        const int32_t *__restrict__ gcol,
                                                        const double *__restrict__ V,
                                                        const double2 *__restrict__ in,
                                                        double2 *__restrict__ out) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)n * nblk) return;
    const int b = (int)(id / n), i = (int)(id - (int64_t)b * n);
    const double2 *x = in + (int64_t)b * n;
    double2 acc = make_double2(0.0, 0.0);
    for (int e = gptr[i]; e < gptr[i + 1]; e++) {
        const double2 v = x[gcol[e]];
        acc.x += V[e] * v.x;
        acc.y += V[e] * v.y;
    }
    out[(int64_t)b * n + i] = acc;
}

}   // namespace

void launch_ldl_solve(const LdlDev &L, const TaskList &tasks, int ntasks, hipStream_t s) {
    hipLaunchKernelGGL(ldl_solve_kernel, dim3(ntasks), dim3(LDL_THREADS), 0, s, L, tasks);
    BEM_LAUNCH_CHECK();
}

void launch_pade_combine(int n, const int32_t *gptr, const int32_t *gcol, const double *Sv,
                         const double2 *cvert, const PadeCoef &pc, const double2 *in,
                         const double2 *sv, int64_t sstride, double2 *out, hipStream_t s) {
    hipLaunchKernelGGL(pade_combine_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, gptr,
                       gcol, Sv, cvert, pc, in, sv, sstride, out);
    BEM_LAUNCH_CHECK();
}

void launch_spmv_real(int n, int nblk, const int32_t *gptr, const int32_t *gcol,
                      const double *V, const double2 *in, double2 *out, hipStream_t s) {
    int64_t work = (int64_t)n * nblk;
    hipLaunchKernelGGL(spmv_real_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s,
                       n, nblk, gptr, gcol, V, in, out);
    BEM_LAUNCH_CHECK();
}

}   // namespace bem

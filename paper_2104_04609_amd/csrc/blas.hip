// Complex FP64 vector kernels of the GMRES solver.  All reductions run in a
// fixed order (per-thread strided sums, then an LDS tree), so repeated runs
// give identical results; no atomics.
#include "bem_internal.h"
#include "blas.h"

namespace bem {

namespace {

constexpr int BT = 256;

// h[i] = sum_k conj(V[i][k]) w[k], one workgroup per basis vector i
__global__ __launch_bounds__(BT) void block_dot_kernel(const double2 *__restrict__ V, int64_t ld,
                                                       const double2 *__restrict__ w, int64_t n,
                                                       double2 *__restrict__ h) {
    __shared__ double sr[BT], si[BT];
    const double2 *v = V + (int64_t)blockIdx.x * ld;
    double ar = 0.0, ai = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += BT) {
        const double2 a = v[k], b = w[k];
        ar += a.x * b.x + a.y * b.y;
        ai += a.x * b.y - a.y * b.x;
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int o = BT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sr[threadIdx.x] += sr[threadIdx.x + o];
            si[threadIdx.x] += si[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) h[blockIdx.x] = make_double2(sr[0], si[0]);
}

// w[k] += sign * sum_{i < m} V[i][k] h[i]   (fixed order in i)
__global__ __launch_bounds__(BT) void block_axpy_kernel(const double2 *__restrict__ V, int64_t ld,
                                                        const double2 *__restrict__ h, int m,
                                                        double sign, double2 *__restrict__ w,
                                                        int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (k >= n) return;
    double ar = 0.0, ai = 0.0;
    for (int i = 0; i < m; i++) {
        const double2 a = V[(int64_t)i * ld + k], b = h[i];
        ar += a.x * b.x - a.y * b.y;
        ai += a.x * b.y + a.y * b.x;
    }
    double2 o = w[k];
    w[k] = make_double2(o.x + sign * ar, o.y + sign * ai);
}

// v /= sqrt(nrm2->x) in place (nrm2 from a block_dot of v with itself)
__global__ __launch_bounds__(BT) void normalize_kernel(double2 *v, const double2 *nrm2,
                                                       int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (k >= n) return;
    const double s = nrm2->x > 0.0 ? 1.0 / sqrt(nrm2->x) : 0.0;
    v[k] = make_double2(v[k].x * s, v[k].y * s);
}

// out = a * x + b * y  (complex scalars)
__global__ __launch_bounds__(BT) void axpby_kernel(double2 a, const double2 *x, double2 b,
                                                   const double2 *y, double2 *out, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (k >= n) return;
    const double2 u = x[k], v = y ? y[k] : make_double2(0.0, 0.0);
    out[k] = make_double2(a.x * u.x - a.y * u.y + b.x * v.x - b.y * v.y,
                          a.x * u.y + a.y * u.x + b.x * v.y + b.y * v.x);
}

// Partial dot products: workgroup (c, i, a) sums conj(V_a[i][k]) w_a[k] over
// chunk c (fixed order: per-thread strided sums, then an LDS tree) into
// part[(a m + i) C + c].
__global__ __launch_bounds__(BT) void dot_partial_kernel(CVecs V, int64_t ld, int m, CVecs w,
                                                         int64_t n, int C,
                                                         double2 *__restrict__ part) {
    __shared__ double sr[BT], si[BT];
    const int c = blockIdx.x, i = blockIdx.y, a = blockIdx.z;
    const double2 *v = V.p[a] + (int64_t)i * ld, *x = w.p[a];
    const int64_t k0 = (int64_t)c * BLAS_DOT_CHUNK;
    const int64_t k1 = k0 + BLAS_DOT_CHUNK < n ? k0 + BLAS_DOT_CHUNK : n;
    double ar = 0.0, ai = 0.0;
    for (int64_t k = k0 + threadIdx.x; k < k1; k += BT) {
        const double2 p = v[k], q = x[k];
        ar += p.x * q.x + p.y * q.y;
        ai += p.x * q.y - p.y * q.x;
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int o = BT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sr[threadIdx.x] += sr[threadIdx.x + o];
            si[threadIdx.x] += si[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[((int64_t)a * m + i) * C + c] = make_double2(sr[0], si[0]);
}

// h_a[i] = sum of the chunks in order; thread a m + i
__global__ __launch_bounds__(BT) void dot_finish_kernel(const double2 *__restrict__ part, int m,
                                                        int C, int A, Vecs h) {
    const int t = blockIdx.x * BT + threadIdx.x;
    if (t >= A * m) return;
    const int a = t / m, i = t - a * m;
    const double2 *p = part + (int64_t)t * C;
    double sx = 0.0, sy = 0.0;
    for (int c = 0; c < C; c++) {
        sx += p[c].x;
        sy += p[c].y;
    }
    h.p[a][i] = make_double2(sx, sy);
}

// w_a[k] += sign * sum_{i < m} V_a[i][k] h_a[i]   (fixed order in i), system blockIdx.y
__global__ __launch_bounds__(BT) void axpy_batch_kernel(CVecs V, int64_t ld, CVecs h, int m,
                                                        double sign, Vecs w, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (k >= n) return;
    const int a = blockIdx.y;
    const double2 *v = V.p[a], *hh = h.p[a];
    double ar = 0.0, ai = 0.0;
    for (int i = 0; i < m; i++) {
        const double2 p = v[(int64_t)i * ld + k], q = hh[i];
        ar += p.x * q.x - p.y * q.y;
        ai += p.x * q.y + p.y * q.x;
    }
    double2 o = w.p[a][k];
    w.p[a][k] = make_double2(o.x + sign * ar, o.y + sign * ai);
}

__global__ __launch_bounds__(BT) void normalize_batch_kernel(Vecs v, CVecs nrm2, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (k >= n) return;
    const int a = blockIdx.y;
    const double q = nrm2.p[a]->x;
    const double sc = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
    v.p[a][k] = make_double2(v.p[a][k].x * sc, v.p[a][k].y * sc);
}

__global__ __launch_bounds__(BT) void copy_batch_kernel(Vecs dst, CVecs src, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * BT + threadIdx.x;
    if (k >= n) return;
    dst.p[blockIdx.y][k] = src.p[blockIdx.y][k];
}

unsigned blocks(int64_t n) { return (unsigned)((n + BT - 1) / BT); }

void check_batch(int A) {
    if (A < 1 || A > BLAS_MAX_BATCH) fail(BEM_E_INVAL, "vector batch out of range");
}

}   // namespace

void blas_block_dot_batch(const CVecs &V, int64_t ld, int m, const CVecs &w, int64_t n,
                          const Vecs &h, int A, double2 *part, hipStream_t s) {
    check_batch(A);
    const int C = (int)blas_dot_chunks(n);
    hipLaunchKernelGGL(dot_partial_kernel, dim3((unsigned)C, (unsigned)m, (unsigned)A), dim3(BT),
                       0, s, V, ld, m, w, n, C, part);
    BEM_LAUNCH_CHECK();
    hipLaunchKernelGGL(dot_finish_kernel, dim3(blocks((int64_t)A * m)), dim3(BT), 0, s, part, m,
                       C, A, h);
    BEM_LAUNCH_CHECK();
}

void blas_block_axpy_batch(const CVecs &V, int64_t ld, const CVecs &h, int m, double sign,
                           const Vecs &w, int64_t n, int A, hipStream_t s) {
    check_batch(A);
    hipLaunchKernelGGL(axpy_batch_kernel, dim3(blocks(n), (unsigned)A), dim3(BT), 0, s, V, ld, h,
                       m, sign, w, n);
    BEM_LAUNCH_CHECK();
}

void blas_normalize_batch(const Vecs &v, const CVecs &nrm2, int64_t n, int A, hipStream_t s) {
    check_batch(A);
    hipLaunchKernelGGL(normalize_batch_kernel, dim3(blocks(n), (unsigned)A), dim3(BT), 0, s, v,
                       nrm2, n);
    BEM_LAUNCH_CHECK();
}

void blas_copy_batch(const Vecs &dst, const CVecs &src, int64_t n, int A, hipStream_t s) {
    check_batch(A);
    hipLaunchKernelGGL(copy_batch_kernel, dim3(blocks(n), (unsigned)A), dim3(BT), 0, s, dst, src,
                       n);
    BEM_LAUNCH_CHECK();
}

void blas_block_dot(const double2 *V, int64_t ld, int m, const double2 *w, int64_t n,
                    double2 *h, hipStream_t s) {
    hipLaunchKernelGGL(block_dot_kernel, dim3(m), dim3(BT), 0, s, V, ld, w, n, h);
    BEM_LAUNCH_CHECK();
}

void blas_block_axpy(const double2 *V, int64_t ld, const double2 *h, int m, double sign,
                     double2 *w, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(block_axpy_kernel, dim3(blocks(n)), dim3(BT), 0, s, V, ld, h, m, sign,
                       w, n);
    BEM_LAUNCH_CHECK();
}

void blas_normalize(double2 *v, const double2 *nrm2, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(normalize_kernel, dim3(blocks(n)), dim3(BT), 0, s, v, nrm2, n);
    BEM_LAUNCH_CHECK();
}

namespace {

// one object's entries of R vectors [R][2N]: sub[r] = [x_r[idx]; x_r[N + idx]]
__global__ __launch_bounds__(256) void gather_halves_kernel(const double2 *__restrict__ x,
                                                            const int32_t *__restrict__ idx,
                                                            int64_t N, int64_t nm,
                                                            double2 *__restrict__ sub) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nm) return;
    const int64_t r = blockIdx.y, v = idx[i];
    sub[2 * nm * r + i] = x[2 * N * r + v];
    sub[2 * nm * r + nm + i] = x[2 * N * r + N + v];
}

__global__ __launch_bounds__(256) void scatter_halves_kernel(const double2 *__restrict__ sub,
                                                             const int32_t *__restrict__ idx,
                                                             int64_t N, int64_t nm,
                                                             double2 *__restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nm) return;
    const int64_t r = blockIdx.y, v = idx[i];
    x[2 * N * r + v] = sub[2 * nm * r + i];
    x[2 * N * r + N + v] = sub[2 * nm * r + nm + i];
}

}   // namespace

void gather_halves(const double2 *x, const int32_t *idx, int64_t N, int64_t nm, int R,
                   double2 *sub, hipStream_t s) {
    hipLaunchKernelGGL(gather_halves_kernel, dim3(blocks(nm), R), dim3(BT), 0, s, x, idx, N, nm,
                       sub);
    BEM_LAUNCH_CHECK();
}

void scatter_halves(const double2 *sub, const int32_t *idx, int64_t N, int64_t nm, int R,
                    double2 *x, hipStream_t s) {
    hipLaunchKernelGGL(scatter_halves_kernel, dim3(blocks(nm), R), dim3(BT), 0, s, sub, idx, N,
                       nm, x);
    BEM_LAUNCH_CHECK();
}

void blas_axpby(double2 a, const double2 *x, double2 b, const double2 *y, double2 *out,
                int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(axpby_kernel, dim3(blocks(n)), dim3(BT), 0, s, a, x, b, y, out, n);
    BEM_LAUNCH_CHECK();
}

}   // namespace bem

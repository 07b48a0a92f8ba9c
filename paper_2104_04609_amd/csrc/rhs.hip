// Plane-wave right-hand side and far-field pattern (FP64).
//
// Right-hand side of the permuted PMCHWT system (Sec. 2.7): the Dirichlet and
// Neumann traces of u_inc = exp(i k d.x) (unit-amplitude plane wave, Sec. 2.1)
// tested with P1 functions, 6-point rule per triangle:
//   f_D,i = int u_inc phi_i,   f_N,i = int i k (d.n) u_inc phi_i.
// Far field from the exterior representation formula (Sec. 2.2) with the
// surface potentials -psi, -phi:
//   F(xhat) = 1/(4 pi) int exp(-i k xhat.y) [-psi(y) - i k (xhat.n_y) phi(y)] dy.
#include <cmath>

#include "bem_internal.h"

namespace bem {

namespace {

constexpr double DUN_A1 = 0.44594849091596488631832925388305;
constexpr double DUN_W1 = 0.22338158967801146569500700843312;
constexpr double DUN_A2 = 0.091576213509770743459571463402202;
constexpr double DUN_W2 = 0.10995174365532186763832632490021;
__host__ __device__ constexpr double qw(int i) { return i < 3 ? DUN_W1 : DUN_W2; }
__host__ __device__ inline double qb(int i, int a) {
    double al = i < 3 ? DUN_A1 : DUN_A2;
    return (a == i % 3) ? (1.0 - 2.0 * al) : al;
}

__device__ inline double2 cexpi(double2 k, double t) {   // exp(i k t)
    double s, c;
    sincos(k.x * t, &s, &c);
    double m = exp(-k.y * t);
    return make_double2(c * m, s * m);
}

// per (wave, triangle): local contributions to f_D and f_N of its 3 vertices
__global__ __launch_bounds__(256) void rhs_local_kernel(const double *__restrict__ geo,
                                                        const double *__restrict__ tst,
                                                        const double *__restrict__ dirs,
                                                        int n_waves, int T, double2 k,
                                                        double2 *__restrict__ loc) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)n_waves * T) return;
    int w = (int)(id / T), t = (int)(id - (int64_t)w * T);
    const double *d = dirs + 3 * w;
    const double *g = geo + (int64_t)GEO_STRIDE * t;
    const double area = tst[TST_STRIDE * t];
    const double dn = d[0] * g[18] + d[1] * g[19] + d[2] * g[20];
    double2 fd[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int j = 0; j < 6; j++) {
        double2 u = cexpi(k, d[0] * g[3 * j] + d[1] * g[3 * j + 1] + d[2] * g[3 * j + 2]);
        for (int a = 0; a < 3; a++) {
            double c = area * qw(j) * qb(j, a);
            fd[a].x += c * u.x;
            fd[a].y += c * u.y;
        }
    }
    double2 *o = loc + 6 * id;
    for (int a = 0; a < 3; a++) {
        o[a] = fd[a];
        // i k (d.n) f_D
        double2 ikd = make_double2(-k.y * dn, k.x * dn);
        o[3 + a] = make_double2(ikd.x * fd[a].x - ikd.y * fd[a].y,
                                ikd.x * fd[a].y + ikd.y * fd[a].x);
    }
}

__global__ __launch_bounds__(256) void rhs_gather_kernel(const double2 *__restrict__ loc,
                                                         const int32_t *__restrict__ star_ptr,
                                                         const int32_t *__restrict__ star_idx,
                                                         int n_waves, int T, int64_t N,
                                                         double2 *__restrict__ f) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)n_waves * N) return;
    int w = (int)(id / N);
    int64_t v = id - (int64_t)w * N;
    double2 a = {0, 0}, b = {0, 0};
    for (int e = star_ptr[v]; e < star_ptr[v + 1]; e++) {
        int ta = star_idx[e];
        int t = ta / 3, l = ta - 3 * t;
        const double2 *o = loc + 6 * ((int64_t)w * T + t);
        a.x += o[l].x;
        a.y += o[l].y;
        b.x += o[3 + l].x;
        b.y += o[3 + l].y;
    }
    f[(int64_t)w * 2 * N + v] = a;
    f[(int64_t)w * 2 * N + N + v] = b;
}

// one workgroup per direction; fixed-order tree reduction in LDS
__global__ __launch_bounds__(256) void far_field_kernel(
    const double *__restrict__ geo, const double *__restrict__ tst,
    const int32_t *__restrict__ tri, const double2 *__restrict__ x, int64_t N, int T,
    const double *__restrict__ dirs, double2 k, double2 *__restrict__ out) {
    __shared__ double2 red[256];
    const double *xh = dirs + 3 * blockIdx.x;
    double2 acc = {0, 0};
    for (int t = threadIdx.x; t < T; t += 256) {
        const double *g = geo + (int64_t)GEO_STRIDE * t;
        const double area = tst[TST_STRIDE * t];
        double2 ps[3], ph[3];
        for (int b = 0; b < 3; b++) {
            int v = tri[3 * t + b];
            ps[b] = x[v];
            ph[b] = x[N + v];
        }
        const double xn = xh[0] * g[18] + xh[1] * g[19] + xh[2] * g[20];
        // -i k (xhat.n)
        const double2 c = make_double2(k.y * xn, -k.x * xn);
        for (int j = 0; j < 6; j++) {
            double2 pj = {0, 0}, fj = {0, 0};
            for (int b = 0; b < 3; b++) {
                pj.x += qb(j, b) * ps[b].x;
                pj.y += qb(j, b) * ps[b].y;
                fj.x += qb(j, b) * ph[b].x;
                fj.y += qb(j, b) * ph[b].y;
            }
            const double proj = xh[0] * g[3 * j] + xh[1] * g[3 * j + 1] + xh[2] * g[3 * j + 2];
            const double2 e = cexpi(make_double2(-k.x, -k.y), proj);   // exp(-i k xhat.y)
            // -psi + c phi
            const double2 v = make_double2(-pj.x + c.x * fj.x - c.y * fj.y,
                                           -pj.y + c.x * fj.y + c.y * fj.x);
            const double wa = area * qw(j);
            acc.x += wa * (e.x * v.x - e.y * v.y);
            acc.y += wa * (e.x * v.y + e.y * v.x);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            red[threadIdx.x].x += red[threadIdx.x + o].x;
            red[threadIdx.x].y += red[threadIdx.x + o].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double s = 0.079577471545947667884441881686257;   // 1/(4 pi)
        out[blockIdx.x] = make_double2(s * red[0].x, s * red[0].y);
    }
}

}   // namespace

void rhs_project(bem_mesh *m, double2 k, const double *dirs, int n, double2 *f,
                 hipStream_t s) {
    const int T = (int)m->T;
    DevBuf<double> d(3 * (size_t)n);
    BEM_HIP(hipMemcpyAsync(d.p, dirs, 3 * n * sizeof(double), hipMemcpyHostToDevice, s));
    DevBuf<double2> loc(6 * (size_t)n * T);
    int64_t work = (int64_t)n * T;
    hipLaunchKernelGGL(rhs_local_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s,
                       m->geo64.p, m->tst.p, d.p, n, T, k, loc.p);
    BEM_LAUNCH_CHECK();
    int64_t work2 = (int64_t)n * m->N;
    hipLaunchKernelGGL(rhs_gather_kernel, dim3((unsigned)((work2 + 255) / 256)), dim3(256), 0,
                       s, loc.p, m->star_ptr.p, m->star_idx.p, n, T, m->N, f);
    BEM_LAUNCH_CHECK();
    BEM_HIP(hipStreamSynchronize(s));   // temporaries are freed on return
}

void far_field_eval(bem_mesh *m, double2 k, const double2 *x, const double *dirs, int n,
                    double2 *out, hipStream_t s) {
    DevBuf<double> d(3 * (size_t)n);
    DevBuf<double2> o(n);
    BEM_HIP(hipMemcpyAsync(d.p, dirs, 3 * n * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(far_field_kernel, dim3(n), dim3(256), 0, s, m->geo64.p, m->tst.p,
                       m->tri_d.p, x, m->N, (int)m->T, d.p, k, o.p);
    BEM_LAUNCH_CHECK();
    BEM_HIP(hipMemcpyAsync(out, o.p, n * sizeof(double2), hipMemcpyDeviceToHost, s));
    BEM_HIP(hipStreamSynchronize(s));
}

}   // namespace bem

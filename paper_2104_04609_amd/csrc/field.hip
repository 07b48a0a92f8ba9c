// Total field at points off the surface (FP64), from a boundary solution
// x = [psi; phi] of the plane wave u_inc = exp(i k_ext d.p).
//
// Representation formulas of Sec. 2.2 with the surface potentials of the
// total field (psi~+ = -psi, phi~+ = -phi outside; psi~- = rho psi,
// phi~- = phi inside, the interior Neumann trace being rho times the
// exterior one):
//   outside every object:  u = u_inc + sum over all triangles of
//       int [ -G_0 psi + (n_y . grad_y G_0) phi ] dy
//   inside object m:       u = int over object m of
//       [ rho_m G_m psi - (n_y . grad_y G_m) phi ] dy
// (k_m, rho_m the object's interior material)
// with n_y . grad_y G(p, y) = ((y - p) . n_y) G (i k r - 1) / r^2; the
// factor (y - p) . n_y = c_sigma - p . n_sigma is constant on a flat
// triangle.  6-point rule per triangle (the sources w |sigma| psi_h and
// w |sigma| phi_h at the rule's points are formed once per call).
//
// Regions: point p is inside object m when the solid angle of m's closed
// surface at p is 4 pi (0 outside); per flat triangle with vertices a, b, c
// relative to p (Van Oosterom and Strackee, 1983):
//   tan(Omega / 2) = a.(b x c) / (|a||b||c| + (a.b)|c| + (a.c)|b| + (b.c)|a|).
// With disjoint objects one pass gives both the total solid angle and, from
// the object-weighted sum, the object that encloses the point.  All sums are
// accumulated in a fixed order (split partials added in split order).
#include <algorithm>
#include <cmath>

#include "bem_internal.h"

namespace bem {

namespace {

constexpr double DUN_A1 = 0.44594849091596488631832925388305;
constexpr double DUN_W1 = 0.22338158967801146569500700843312;
constexpr double DUN_A2 = 0.091576213509770743459571463402202;
constexpr double DUN_W2 = 0.10995174365532186763832632490021;
__device__ constexpr double qw(int i) { return i < 3 ? DUN_W1 : DUN_W2; }
__device__ inline double qb(int i, int a) {
    const double al = i < 3 ? DUN_A1 : DUN_A2;
    return (a == i % 3) ? (1.0 - 2.0 * al) : al;
}

constexpr double INV4PI = 0.079577471545947667884441881686257;
constexpr double TWO_PI = 6.283185307179586476925286766559;
constexpr double INV2PI = 0.15915494309189533576888376337251;

// sin and cos of 2 pi t from a table of e^{2 pi i n / 256} (n = nearest
// integer to 256 t) and the Taylor series of the remainder 2 pi f, |f| <=
// 1/512 (terms beyond x^6 below 4e-18), joined by one complex product
__device__ __forceinline__ void sincos_turns(double t, double &s, double &c,
                                             const double2 *__restrict__ tab) {
    const double n = __builtin_rint(256.0 * t);
    const double x = __builtin_fma(-0.00390625, n, t) * TWO_PI;
    const double x2 = x * x;
    const double sn = __builtin_fma(__builtin_fma(x2, 1.0 / 120.0, -1.0 / 6.0), x2, 1.0) * x;
    const double cs =
        __builtin_fma(__builtin_fma(__builtin_fma(x2, -1.0 / 720.0, 1.0 / 24.0), x2, -0.5), x2, 1.0);
    const double2 e = tab[((int64_t)n) & 255];
    c = __builtin_fma(e.x, cs, -e.y * sn);
    s = __builtin_fma(e.y, cs, e.x * sn);
}

// 1/sqrt(x): hardware estimate and two Newton steps
__device__ __forceinline__ double rsq64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * __builtin_fma(-h * y, y, 1.5);
    y = y * __builtin_fma(-h * y, y, 1.5);
    return y;
}

// per triangle: the 6 rule points, w |sigma| psi_h and w |sigma| phi_h there
constexpr int SRC_STRIDE = 42;   // [0,18) points, [18,30) s_psi, [30,42) s_phi
constexpr int FT = 64;           // triangles per LDS tile
constexpr int FS = 48;           // tile doubles per triangle: SRC + normal, c, object

__global__ __launch_bounds__(256) void field_sources_kernel(
    const double *__restrict__ P, const int32_t *__restrict__ tri,
    const double *__restrict__ tst, const double2 *__restrict__ x, int64_t N, int T,
    double *__restrict__ src) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double v[3][3];
    double2 ps[3], ph[3];
    for (int b = 0; b < 3; b++) {
        const int vi = tri[3 * t + b];
        for (int c = 0; c < 3; c++) v[b][c] = P[3 * vi + c];
        ps[b] = x[vi];
        ph[b] = x[N + vi];
    }
    const double area = tst[TST_STRIDE * t];
    double *o = src + (int64_t)SRC_STRIDE * t;
    for (int q = 0; q < 6; q++) {
        const double wa = qw(q) * area;
        double pr = 0, pi = 0, fr = 0, fi = 0;
        for (int b = 0; b < 3; b++) {
            const double l = qb(q, b);
            pr += l * ps[b].x;
            pi += l * ps[b].y;
            fr += l * ph[b].x;
            fi += l * ph[b].y;
        }
        for (int c = 0; c < 3; c++)
            o[3 * q + c] = qb(q, 0) * v[0][c] + qb(q, 1) * v[1][c] + qb(q, 2) * v[2][c];
        o[18 + 2 * q] = wa * pr;
        o[18 + 2 * q + 1] = wa * pi;
        o[30 + 2 * q] = wa * fr;
        o[30 + 2 * q + 1] = wa * fi;
    }
}

constexpr int WS = 10;   // winding tile doubles per triangle: 3 vertices, object

// Work split over trial-triangle ranges (blockIdx.y): each (split, point)
// writes its partial sums; the reduction kernels add the splits in order.

// partial solid angles of all triangles of the split at each point:
// [0] sum Omega_t, [1] sum Omega_t (object_t + 1)
__global__ __launch_bounds__(256) void winding_kernel(
    const double *__restrict__ P, const int32_t *__restrict__ tri,
    const int32_t *__restrict__ tobj, int T, int split_len, const double *__restrict__ pts,
    int64_t n, double *__restrict__ part) {
    __shared__ double tile[FT * WS];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t pp = p < n ? p : 0;
    const double px = pts[3 * pp], py = pts[3 * pp + 1], pz = pts[3 * pp + 2];
    const int t0 = blockIdx.y * split_len, t1 = min(T, t0 + split_len);
    double om = 0.0, ow = 0.0;
    for (int base = t0; base < t1; base += FT) {
        const int cnt = min(FT, t1 - base);
        __syncthreads();
        for (int idx = threadIdx.x; idx < cnt * WS; idx += blockDim.x) {
            const int sl = idx / WS, f = idx - sl * WS;
            const int64_t t = base + sl;
            tile[idx] = f < 9 ? P[3 * tri[3 * t + f / 3] + f % 3] : (double)(tobj[t] + 1);
        }
        __syncthreads();
        for (int sl = 0; sl < cnt; sl++) {
            const double *v = tile + sl * WS;
            const double a0 = v[0] - px, a1 = v[1] - py, a2 = v[2] - pz;
            const double b0 = v[3] - px, b1 = v[4] - py, b2 = v[5] - pz;
            const double c0 = v[6] - px, c1 = v[7] - py, c2 = v[8] - pz;
            const double la = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
            const double lb = sqrt(b0 * b0 + b1 * b1 + b2 * b2);
            const double lc = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
            const double num = a0 * (b1 * c2 - b2 * c1) + a1 * (b2 * c0 - b0 * c2) +
                               a2 * (b0 * c1 - b1 * c0);
            const double den = la * lb * lc + (a0 * b0 + a1 * b1 + a2 * b2) * lc +
                               (a0 * c0 + a1 * c1 + a2 * c2) * lb +
                               (b0 * c0 + b1 * c1 + b2 * c2) * la;
            const double o = 2.0 * atan2(num, den);
            om += o;
            ow += o * v[9];
        }
    }
    if (p < n) {
        part[2 * ((int64_t)blockIdx.y * n + p)] = om;
        part[2 * ((int64_t)blockIdx.y * n + p) + 1] = ow;
    }
}

// Closed disjoint surfaces: the total solid angle is 4 pi inside one object
// and 0 outside all; inside object m the object-weighted sum is (m + 1) times
// the total, since every other surface subtends 0.
__global__ __launch_bounds__(256) void region_kernel(const double *__restrict__ part, int nsplit,
                                                     int64_t n, int nobj,
                                                     int32_t *__restrict__ region) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double om = 0.0, ow = 0.0;
    for (int sp = 0; sp < nsplit; sp++) {
        om += part[2 * ((int64_t)sp * n + p)];
        ow += part[2 * ((int64_t)sp * n + p) + 1];
    }
    int r = 0;
    if (fabs(om) > TWO_PI) r = min(nobj, max(1, (int)lround(ow / om)));
    region[p] = r;
}

// partial single- and double-layer sums of the split's triangles at each
// point, with the wavenumber and the triangles of the point's region
// Three waves per SIMD (measured against two: 5 % faster; four: 2.6x slower).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void field_kernel(
    const double *__restrict__ src, const double *__restrict__ geo,
    const int32_t *__restrict__ tobj, int T, int split_len, const double *__restrict__ pts,
    const int32_t *__restrict__ region, int64_t n, double2 k0, const double *__restrict__ omat,
    double *__restrict__ part) {
    __shared__ double tile[FT * FS];
    __shared__ double2 etab[256];   // e^{2 pi i n / 256}
    for (int i = threadIdx.x; i < 256; i += blockDim.x) {
        double sn, cs;
        sincos(i * (TWO_PI / 256.0), &sn, &cs);
        etab[i] = make_double2(cs, sn);
    }
    // (the first tile's barrier orders these writes before any read)
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t pp = p < n ? p : 0;
    const double px = pts[3 * pp], py = pts[3 * pp + 1], pz = pts[3 * pp + 2];
    const int reg = region[pp];
    const bool ext = reg == 0;
    // interior material of the enclosing object: omat[object] = (Re k, Im k, rho)
    const double2 k = ext ? k0 : make_double2(omat[3 * (reg - 1)], omat[3 * (reg - 1) + 1]);
    const double krev = k.x * INV2PI;
    const int t0 = blockIdx.y * split_len, t1 = min(T, t0 + split_len);
    double sr = 0, si = 0, dr = 0, di = 0;
    for (int base = t0; base < t1; base += FT) {
        const int cnt = min(FT, t1 - base);
        __syncthreads();
        for (int idx = threadIdx.x; idx < cnt * FS; idx += blockDim.x) {
            const int sl = idx / FS, f = idx - sl * FS;
            const int64_t t = base + sl;
            double v;
            if (f < SRC_STRIDE) v = src[SRC_STRIDE * t + f];
            else if (f < SRC_STRIDE + 3) v = geo[GEO_STRIDE * t + 18 + (f - SRC_STRIDE)];
            else if (f == SRC_STRIDE + 3) v = geo[GEO_STRIDE * t + 21];
            else v = (double)tobj[t];
            tile[idx] = v;
        }
        __syncthreads();
        for (int sl = 0; sl < cnt; sl++) {
            const double *s = tile + sl * FS;
            if (!ext && (int)s[SRC_STRIDE + 4] != reg - 1) continue;
            // (y - p) . n_sigma, constant on the flat triangle
            const double dn = s[SRC_STRIDE + 3] -
                              (px * s[SRC_STRIDE] + py * s[SRC_STRIDE + 1] + pz * s[SRC_STRIDE + 2]);
            double fr = 0, fi = 0;
            for (int q = 0; q < 6; q++) {
                const double ex = s[3 * q] - px, ey = s[3 * q + 1] - py, ez = s[3 * q + 2] - pz;
                const double r2 = ex * ex + ey * ey + ez * ez;
                const double ri = rsq64(r2);
                const double r = r2 * ri;
                double sn, cs;
                sincos_turns(krev * r, sn, cs, etab);
                const double mag = (k.y != 0.0 ? exp(-k.y * r) : 1.0) * ri;
                const double Gr = cs * mag, Gi = sn * mag;     // 4 pi G
                // 4 pi G (i k r - 1) / r^2
                const double tr = -1.0 - k.y * r, ti = k.x * r;
                const double ri2 = ri * ri;   // (= 1 / r2)
                const double Fr = (Gr * tr - Gi * ti) * ri2, Fi = (Gr * ti + Gi * tr) * ri2;
                const double ar = s[18 + 2 * q], ai = s[18 + 2 * q + 1];
                const double br = s[30 + 2 * q], bi = s[30 + 2 * q + 1];
                sr += Gr * ar - Gi * ai;
                si += Gr * ai + Gi * ar;
                fr += Fr * br - Fi * bi;
                fi += Fr * bi + Fi * br;
            }
            dr += dn * fr;
            di += dn * fi;
        }
    }
    if (p < n) {
        double *o = part + 4 * ((int64_t)blockIdx.y * n + p);
        o[0] = sr;
        o[1] = si;
        o[2] = dr;
        o[3] = di;
    }
}

// splits added in order; coefficients of the region; incident wave outside
__global__ __launch_bounds__(256) void field_reduce_kernel(
    const double *__restrict__ part, int nsplit, const double *__restrict__ pts,
    const int32_t *__restrict__ region, int64_t n, double2 k0, const double *__restrict__ omat,
    double dx, double dy, double dz, double2 *__restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double sr = 0, si = 0, dr = 0, di = 0;
    for (int sp = 0; sp < nsplit; sp++) {
        const double *o = part + 4 * ((int64_t)sp * n + p);
        sr += o[0];
        si += o[1];
        dr += o[2];
        di += o[3];
    }
    double ur, ui;
    const int reg = region[p];
    if (reg == 0) {
        const double dp = dx * pts[3 * p] + dy * pts[3 * p + 1] + dz * pts[3 * p + 2];
        double sn, cs;
        sincos(k0.x * dp, &sn, &cs);
        const double a = exp(-k0.y * dp);
        ur = a * cs + INV4PI * (dr - sr);
        ui = a * sn + INV4PI * (di - si);
    } else {
        const double rho = omat[3 * (reg - 1) + 2];
        ur = INV4PI * (rho * sr - dr);
        ui = INV4PI * (rho * si - di);
    }
    out[p] = make_double2(ur, ui);
}

}   // namespace

void field_eval(bem_mesh *m, double2 k0, double2 k1, double rho, const double *dir,
                const double2 *x, const double *pts, int64_t n, double2 *out, int32_t *region,
                hipStream_t s, const ObjMaterials *om) {
    if (n == 0) return;
    const int T = (int)m->T;
    if (!m->P_d.p) m->P_d.upload(m->P);
    std::vector<double> mat(3 * (size_t)m->nobj);
    for (int o = 0; o < m->nobj; o++) {
        const double2 ko = om ? om->k[o] : k1;
        mat[3 * o] = ko.x;
        mat[3 * o + 1] = ko.y;
        mat[3 * o + 2] = om ? om->rho[o] : rho;
    }
    DevBuf<double> matd;
    matd.upload(mat);
    const unsigned pb = (unsigned)((n + 255) / 256);
    // enough workgroups to fill the device (about 2048), splits of >= 4 tiles
    const int max_split = std::max(1, T / (4 * FT));
    const int nsplit = (int)std::min<int64_t>(max_split, std::max<int64_t>(1, (2048 + pb - 1) / pb));
    const int split_len = (T + nsplit - 1) / nsplit;
    DevBuf<double> src((size_t)SRC_STRIDE * T);
    DevBuf<double> part((size_t)nsplit * n * 4);
    DevBuf<int32_t> reg_own;
    int32_t *reg = region;
    if (!reg) {
        reg_own.alloc((size_t)n);
        reg = reg_own.p;
    }
    hipLaunchKernelGGL(field_sources_kernel, dim3((T + 255) / 256), dim3(256), 0, s, m->P_d.p,
                       m->tri_d.p, m->tst.p, x, m->N, T, src.p);
    BEM_LAUNCH_CHECK();
    {
        Timer tm("field_winding", s);
        hipLaunchKernelGGL(winding_kernel, dim3(pb, (unsigned)nsplit), dim3(256), 0, s, m->P_d.p,
                           m->tri_d.p, m->tobj_d.p, T, split_len, pts, n, part.p);
        BEM_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(region_kernel, dim3(pb), dim3(256), 0, s, part.p, nsplit, n, m->nobj, reg);
    BEM_LAUNCH_CHECK();
    {
        Timer tm("field_eval", s);
        hipLaunchKernelGGL(field_kernel, dim3(pb, (unsigned)nsplit), dim3(256), 0, s, src.p,
                           m->geo64.p, m->tobj_d.p, T, split_len, pts, reg, n, k0, matd.p,
                           part.p);
        BEM_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(field_reduce_kernel, dim3(pb), dim3(256), 0, s, part.p, nsplit, pts, reg, n,
                       k0, matd.p, dir[0], dir[1], dir[2], out);
    BEM_LAUNCH_CHECK();
    BEM_HIP(hipStreamSynchronize(s));   // src, part and the own region buffer are released on return
}

}   // namespace bem

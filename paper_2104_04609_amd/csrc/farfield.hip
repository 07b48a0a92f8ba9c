// Matrix-free Galerkin matvec of the permuted PMCHWT operator (Sec. 2.7):
//
//   y1 = (V_0 + rho V_1) psi - (K_0 + K_1) phi
//   y2 = (K'_0 + K'_1) psi + (D_0 + D_1 / rho) phi
//
// with the operators of Sec. 2.2 (D in Maue form) on P1 functions (Sec. 2.3).
// For every test triangle tau and every trial triangle sigma that shares no
// vertex with tau the 6x6 tensor 6-point rule is applied here; pairs sharing
// a vertex (coinciding, edge- or vertex-adjacent) are integrated entirely by
// the FP64 near-field CSR operator, built once per wavenumber pair.
//
// Per point pair (x in tau, y in sigma), r = |x - y|, E_m = e^{i k_m r},
// G_m = E_m/r and F_m = G_m (i k_m r - 1)/r^2 (the 1/4pi is applied once at
// the end):
//   G_V = G_0 + rho G_1       (single layer, row 1)
//   G_W = G_0 + G_1 / rho     (hypersingular curl-curl part, row 2)
//   G_N = k_0^2 G_0 + k_1^2 G_1 / rho   (hypersingular normal part, row 2)
//   F   = F_0 + F_1 = (i (k_0 E_0 + k_1 E_1) - G_0 - G_1) / r^2
//   acc1(x) += G_V s_psi(y) - F (y - x).n_y s_phi(y)
//   acc2(x) += F (x - y).n_x s_psi(y) - G_N (n_x.n_y) s_phi(y)
//   A_tau   += w_x w_y G_W sC_sigma        (curl term, contracted per pair)
// s_psi(y) = w_y |sigma| psi_h(y), sC_sigma = |sigma| curl(phi_h) on sigma.
// Factors constant over the points y of one trial triangle are taken out of
// the y sum: (y - x).n_y = c_sigma - x.n_sigma (per x), (x - y).n_x =
// c_tau - y.n_tau (per y, folded into s_psi), and k_0^2 (n_x.n_y) per triangle pair.
// Interior terms (index 1) are masked out for triangles of different objects.
// The Mueller operator (Sec. 2.2) is the same sum with the interior terms
// negated; its identity part lives in the near-field operator, so the pair
// kernels only see the sign, folded into the launch coefficients.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <queue>
#include <type_traits>
#include <utility>

#include "bem_internal.h"

namespace bem {

namespace {

constexpr int FF_BLOCK = 256;   // largest workgroup (test triangles per workgroup)
constexpr int FF_TILE = 32;     // trial triangles per LDS tile
constexpr int SRC = GEO_STRIDE + DYN_STRIDE + 4;   // + object id, 3 vertex ids

// 6-point rule (Dunavant, degree 4): orbits (1-2a, a, a); compile-time
// constants so that the unrolled point loops fold them.
constexpr double DUN_A1 = 0.44594849091596488631832925388305;
constexpr double DUN_W1 = 0.22338158967801146569500700843312;
constexpr double DUN_A2 = 0.091576213509770743459571463402202;
constexpr double DUN_W2 = 0.10995174365532186763832632490021;
__host__ __device__ constexpr double qw(int i) { return i < 3 ? DUN_W1 : DUN_W2; }
__host__ __device__ constexpr double qb(int i, int a) {
    return (a == i % 3) ? (1.0 - 2.0 * (i < 3 ? DUN_A1 : DUN_A2)) : (i < 3 ? DUN_A1 : DUN_A2);
}
// FP32 roundings of the weight products, read with a point index j that is
// uniform over the wavefront (a loop counter) through the scalar cache, so
// that no FP64 arithmetic or selects run per point pair:
// kQW2[6 j + i] = (float)(qw(i) qw(j)), kQWB[3 j + a] = (float)(qw(j) qb(j, a)).
#define BEM_QW2_ROW(j)                                                                       \
    (float)(qw(0) * qw(j)), (float)(qw(1) * qw(j)), (float)(qw(2) * qw(j)),                 \
        (float)(qw(3) * qw(j)), (float)(qw(4) * qw(j)), (float)(qw(5) * qw(j))
#define BEM_QWB_ROW(j) (float)(qw(j) * qb(j, 0)), (float)(qw(j) * qb(j, 1)), (float)(qw(j) * qb(j, 2))
__constant__ float kQW2[36] = {BEM_QW2_ROW(0), BEM_QW2_ROW(1), BEM_QW2_ROW(2),
                               BEM_QW2_ROW(3), BEM_QW2_ROW(4), BEM_QW2_ROW(5)};
__constant__ float kQWB[18] = {BEM_QWB_ROW(0), BEM_QWB_ROW(1), BEM_QWB_ROW(2),
                               BEM_QWB_ROW(3), BEM_QWB_ROW(4), BEM_QWB_ROW(5)};
#undef BEM_QW2_ROW
#undef BEM_QWB_ROW

// ---------------------------------------------------------------- math
template <class R> struct Math;

template <> struct Math<float> {
    // sin/cos of 2 pi t: hardware v_sin/v_cos take revolutions.  With FR the
    // argument is first reduced exactly to its fractional part; without it
    // the caller guarantees |t| < 256 revolutions, inside which the hardware
    // reduction gives the same values (sin may differ by a last-bit rounding
    // near its zeros).
    template <bool FR>
    static __device__ __forceinline__ void sincos_rev(float t, float &s, float &c) {
        const float f = FR ? __builtin_amdgcn_fractf(t) : t;
        s = __builtin_amdgcn_sinf(f);
        c = __builtin_amdgcn_cosf(f);
    }
    static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float exp2(float x) { return __builtin_amdgcn_exp2f(x); }
};

template <> struct Math<double> {
    // sin/cos of 2 pi t for moderate |t|: t = n/4 + f, |f| <= 1/8, then
    // Taylor series of sin and cos on [-pi/4, pi/4] (truncation < 5e-17) and
    // the quadrant rotation by n.
    template <bool FR>
    static __device__ __forceinline__ void sincos_rev(double t, double &s, double &c) {
        double n = __builtin_rint(4.0 * t);
        double f = __builtin_fma(-0.25, n, t);
        double x = f * 6.283185307179586476925286766559;
        double x2 = x * x;
        double ps = 1.0 / 1307674368000.0;           // 1/15!
        ps = __builtin_fma(ps, -x2, 1.0 / 6227020800.0);    // 1/13!
        ps = __builtin_fma(ps, -x2, 1.0 / 39916800.0);      // 1/11!
        ps = __builtin_fma(ps, -x2, 1.0 / 362880.0);        // 1/9!
        ps = __builtin_fma(ps, -x2, 1.0 / 5040.0);          // 1/7!
        ps = __builtin_fma(ps, -x2, 1.0 / 120.0);           // 1/5!
        ps = __builtin_fma(ps, -x2, 1.0 / 6.0);             // 1/3!
        ps = __builtin_fma(ps, -x2, 1.0);
        double sn = ps * x;
        double pc = 1.0 / 20922789888000.0;          // 1/16!
        pc = __builtin_fma(pc, -x2, 1.0 / 87178291200.0);   // 1/14!
        pc = __builtin_fma(pc, -x2, 1.0 / 479001600.0);     // 1/12!
        pc = __builtin_fma(pc, -x2, 1.0 / 3628800.0);       // 1/10!
        pc = __builtin_fma(pc, -x2, 1.0 / 40320.0);         // 1/8!
        pc = __builtin_fma(pc, -x2, 1.0 / 720.0);           // 1/6!
        pc = __builtin_fma(pc, -x2, 1.0 / 24.0);            // 1/4!
        pc = __builtin_fma(pc, -x2, 0.5);                   // 1/2!
        double cs = __builtin_fma(pc, -x2, 1.0);
        int q = ((int)n) & 3;
        double s0 = (q & 1) ? cs : sn;
        double c0 = (q & 1) ? sn : cs;
        s = (q & 2) ? -s0 : s0;
        c = ((q + 1) & 2) ? -c0 : c0;
    }
    // sin/cos of 2 pi t with a table of e^{2 pi i n / 256}: t = n/256 + f,
    // |f| <= 1/512, so |2 pi f| <= 0.0123 and short Taylor series suffice
    // (truncation x^7/7! < 4e-18, x^8/8! < 2e-20); then one complex product.
    static __device__ __forceinline__ void sincos_tab(double t, double &s, double &c,
                                                      const double2 *tab) {
        const double n = __builtin_rint(256.0 * t);
        const double f = __builtin_fma(-0.00390625, n, t);
        const double x = f * 6.283185307179586476925286766559;
        const double x2 = x * x;
        double ps = __builtin_fma(x2, 1.0 / 120.0, -1.0 / 6.0);
        ps = __builtin_fma(ps, x2, 1.0);
        const double sn = ps * x;
        double pc = __builtin_fma(x2, -1.0 / 720.0, 1.0 / 24.0);
        pc = __builtin_fma(pc, x2, -0.5);
        const double cs = __builtin_fma(pc, x2, 1.0);
        const double2 e = tab[((int)n) & 255];
        c = __builtin_fma(e.x, cs, -e.y * sn);
        s = __builtin_fma(e.y, cs, e.x * sn);
    }
    // 1/sqrt(x): hardware estimate refined by two Newton steps
    static __device__ __forceinline__ double rsq(double x) {
        double y = __builtin_amdgcn_rsq(x);
        double h = 0.5 * x;
        y = y * __builtin_fma(-h * y, y, 1.5);
        y = y * __builtin_fma(-h * y, y, 1.5);
        return y;
    }
    static __device__ __forceinline__ double exp2(double x) { return ::exp2(x); }
};

__device__ __forceinline__ float fmac(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}
__device__ __forceinline__ double fmac(double a, double b, double c) {
    return __builtin_fma(a, b, c);
}

// Interior coefficients of one object (material k_1, rho of that object).
constexpr int INT_COEFS = 9;
template <class R> struct Int {
    R krev1;                 // Re k_1 / (2 pi)
    R k1r, k1i;              // k_1
    R kdec1;                 // -Im k_1 * log2(e)
    R rho, irho;
    R n10r, n10i;            // k_1^2 / (rho k_0^2)
    R ns1;                   // -s_1
};

// Wavenumber-dependent coefficients of one launch.  Kernels for several
// objects take the interior part of each trial triangle's object from a
// per-object table instead of `in`.
template <class R> struct Coef {
    R krev0;                 // Re k_0 / (2 pi)
    R k0r, k0i;              // k_0
    R kdec0;                 // -Im k_0 * log2(e)
    R n0r, n0i;              // k_0^2
    Int<R> in;
};

// interior coefficients for a trial triangle of object `obj` (uniform over
// the wave: every lane reads the same trial triangle)
template <bool MULTI, class R>
__device__ __forceinline__ Int<R> interior(const Coef<R> &cf, const Int<R> *__restrict__ itab,
                                           R obj) {
    if constexpr (MULTI) {
        const int ob = __builtin_amdgcn_readfirstlane((int)obj);
        return itab[ob];
    } else {
        return cf.in;
    }
}

// ------------------------------------------------------------ source gather
template <class R>
__global__ __launch_bounds__(256) void source_gather_kernel(
    const int32_t *__restrict__ tri, const double *__restrict__ tst,
    const double2 *__restrict__ x, int64_t N, int T, R *__restrict__ dyn) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= T) return;
    double2 ps[3], ph[3];
    for (int b = 0; b < 3; b++) {
        int v = tri[3 * s + b];
        ps[b] = x[v];
        ph[b] = x[N + v];
    }
    const double area = tst[TST_STRIDE * s];
    R *out = dyn + (int64_t)DYN_STRIDE * s;
    for (int j = 0; j < 6; j++) {
        double wa = qw(j) * area;
        double pr = 0, pi = 0, fr = 0, fi = 0;
        for (int b = 0; b < 3; b++) {
            pr += qb(j, b) * ps[b].x;
            pi += qb(j, b) * ps[b].y;
            fr += qb(j, b) * ph[b].x;
            fi += qb(j, b) * ph[b].y;
        }
        out[2 * j] = (R)(wa * pr);
        out[2 * j + 1] = (R)(wa * pi);
        out[12 + 2 * j] = (R)(wa * fr);
        out[12 + 2 * j + 1] = (R)(wa * fi);
    }
    for (int c = 0; c < 3; c++) {
        double cr = 0, ci = 0;
        for (int b = 0; b < 3; b++) {
            double cu = tst[TST_STRIDE * s + 1 + 3 * b + c];
            cr += cu * ph[b].x;
            ci += cu * ph[b].y;
        }
        out[24 + 2 * c] = (R)(area * cr);
        out[24 + 2 * c + 1] = (R)(area * ci);
    }
}

// ------------------------------------------------------- fused pair kernel
// FP32: per-tile FP64 row sums live in LDS (one column per thread), which
// keeps the kernel within 168 VGPRs, i.e. 3 waves per SIMD.
constexpr int FF_ROWS = ROW_STRIDE + 6;   // 12 row sums + 6 curl sums
template <class R> constexpr int ff_waves() { return std::is_same<R, float>::value ? 3 : 2; }

template <class R, bool CK0, bool CK1, bool MULTI, bool FR>
__global__ __launch_bounds__(FF_BLOCK) __attribute__((amdgpu_waves_per_eu(ff_waves<R>())))
void farfield_kernel(
    const R *__restrict__ geo, const R *__restrict__ dyn,
    const int32_t *__restrict__ tobj, const int32_t *__restrict__ tri, int T,
    int split_len, Coef<R> cf, const Int<R> *__restrict__ itab,
    double *__restrict__ partial) {
    using MT = Math<R>;
    constexpr bool F32 = std::is_same<R, float>::value;
    __shared__ R tile[FF_TILE * SRC];
    // FP64: e^{2 pi i n / 256}, n < 256, for the table-based sin/cos
    __shared__ double2 etab[F32 ? 1 : 256];
    extern __shared__ double sums[];   // FP32: [FF_ROWS][blockDim.x] (dynamic)
    const int nthr = blockDim.x;
    const int tau = blockIdx.x * nthr + threadIdx.x;
    const int split = blockIdx.y;
    if constexpr (!F32) {
        for (int n = threadIdx.x; n < 256; n += nthr) {
            double sn, cs;
            MT::template sincos_rev<true>(n * 0.00390625, sn, cs);
            etab[n] = make_double2(cs, sn);
        }
        // the first tile's barrier orders these writes before any read
    }
    const int s_begin = split * split_len;
    const int s_end = min(T, s_begin + split_len);
    const bool active = tau < T;
    const int tt = active ? tau : 0;

    R px[6], py[6], pz[6];
    for (int i = 0; i < 6; i++) {
        px[i] = geo[GEO_STRIDE * tt + 3 * i];
        py[i] = geo[GEO_STRIDE * tt + 3 * i + 1];
        pz[i] = geo[GEO_STRIDE * tt + 3 * i + 2];
    }
    const R ntx = geo[GEO_STRIDE * tt + 18], nty = geo[GEO_STRIDE * tt + 19],
            ntz = geo[GEO_STRIDE * tt + 20], ct = geo[GEO_STRIDE * tt + 21];
    const R ot = MULTI ? (R)tobj[tt] : (R)0;
    // vertex ids as R (exact: N < 2^24) for the adjacency test
    const R tv0 = (R)tri[3 * tt], tv1 = (R)tri[3 * tt + 1], tv2 = (R)tri[3 * tt + 2];

    R a1r[6], a1i[6], a2r[6], a2i[6];
    R Ar[3], Ai[3];
    for (int i = 0; i < 6; i++) a1r[i] = a1i[i] = a2r[i] = a2i[i] = 0;
    for (int c = 0; c < 3; c++) Ar[c] = Ai[c] = 0;
    // FP64 sums: rows c = 0..11 (row 1 / row 2, test vertex, re/im), then the
    // 6 curl sums; in LDS for FP32, in registers for FP64
    double regsum[F32 ? 1 : FF_ROWS];
    auto sum_add = [&](int c, double v) {
        if constexpr (F32) sums[c * nthr + threadIdx.x] += v;
        else regsum[c] += v;
    };
    if constexpr (F32) {
        for (int c = 0; c < FF_ROWS; c++) sums[c * nthr + threadIdx.x] = 0;
    } else {
        for (int c = 0; c < FF_ROWS; c++) regsum[c] = 0;
    }

    auto flush = [&]() {
        for (int a = 0; a < 3; a++) {
            double r1r = 0, r1i = 0, r2r = 0, r2i = 0;
            for (int i = 0; i < 6; i++) {
                double wb = qw(i) * qb(i, a);
                r1r += wb * (double)a1r[i];
                r1i += wb * (double)a1i[i];
                r2r += wb * (double)a2r[i];
                r2i += wb * (double)a2i[i];
            }
            sum_add(2 * a, r1r);
            sum_add(2 * a + 1, r1i);
            sum_add(6 + 2 * a, r2r);
            sum_add(6 + 2 * a + 1, r2i);
        }
        for (int c = 0; c < 3; c++) {
            sum_add(ROW_STRIDE + 2 * c, (double)Ar[c]);
            sum_add(ROW_STRIDE + 2 * c + 1, (double)Ai[c]);
            Ar[c] = Ai[c] = 0;
        }
        for (int i = 0; i < 6; i++) a1r[i] = a1i[i] = a2r[i] = a2i[i] = 0;
    };

    for (int base = s_begin; base < s_end; base += FF_TILE) {
        const int cnt = min(FF_TILE, s_end - base);
        __syncthreads();
        for (int idx = threadIdx.x; idx < cnt * SRC; idx += nthr) {
            int s = idx / SRC, f = idx - s * SRC;
            R v;
            if (f < GEO_STRIDE) v = geo[(int64_t)GEO_STRIDE * (base + s) + f];
            else if (f < GEO_STRIDE + DYN_STRIDE)
                v = dyn[(int64_t)DYN_STRIDE * (base + s) + (f - GEO_STRIDE)];
            else if (f == GEO_STRIDE + DYN_STRIDE) v = MULTI ? (R)tobj[base + s] : (R)0;
            else v = (R)tri[3 * (base + s) + (f - GEO_STRIDE - DYN_STRIDE - 1)];
            tile[idx] = v;
        }
        __syncthreads();
        for (int s = 0; s < cnt; s++) {
            const R *src = &tile[s * SRC];
            {
                const R *sv = src + GEO_STRIDE + DYN_STRIDE + 1;
                const bool adj = sv[0] == tv0 || sv[0] == tv1 || sv[0] == tv2 ||
                                 sv[1] == tv0 || sv[1] == tv1 || sv[1] == tv2 ||
                                 sv[2] == tv0 || sv[2] == tv1 || sv[2] == tv2;
                if (adj) continue;   // includes sigma == tau: near field
            }
            const R nsx = src[18], nsy = src[19], nsz = src[20], cs = src[21];
            const R m1 = MULTI ? (src[GEO_STRIDE + DYN_STRIDE] == ot ? (R)1 : (R)0) : (R)1;
            const Int<R> c1 = interior<MULTI>(cf, itab, src[GEO_STRIDE + DYN_STRIDE]);
            const R nn = ntx * nsx + nty * nsy + ntz * nsz;
            // factor of the G_N term pulled out of the j sum: k_0^2 (n_x . n_y)
            const R gnr = cf.n0r * nn, gni = cf.n0i * nn;
            R dny[6];
            for (int i = 0; i < 6; i++)
                dny[i] = cs - (px[i] * nsx + py[i] * nsy + pz[i] * nsz);
            // per test point: sums over j of F s_phi and (G_0 + n10 G_1) s_phi,
            // scaled by (y - x).n_y resp. k_0^2 (n_x . n_y) after the j loop
            R qr[6], qi[6], nr[6], ni[6];
            for (int i = 0; i < 6; i++) qr[i] = qi[i] = nr[i] = ni[i] = 0;
            R gwr = 0, gwi = 0;
            // j outer and not unrolled: few values live across the loop and
            // a compact body (i unrolled inside)
#pragma unroll 1
            for (int j = 0; j < 6; j++) {
                const R yx = src[3 * j], yy = src[3 * j + 1], yz = src[3 * j + 2];
                const R spr = src[GEO_STRIDE + 2 * j], spi = src[GEO_STRIDE + 2 * j + 1];
                const R sfr = src[GEO_STRIDE + 12 + 2 * j], sfi = src[GEO_STRIDE + 12 + 2 * j + 1];
                // (x_i - y_j).n_x s_psi(y_j) = (c_tau - y_j.n_x) s_psi(y_j)
                const R dnx = ct - (yx * ntx + yy * nty + yz * ntz);
                const R spxr = dnx * spr, spxi = dnx * spi;
                const R wj = (R)qw(j);
#pragma unroll
                for (int i = 0; i < 6; i++) {
                    const R dx = yx - px[i];
                    const R dy = yy - py[i];
                    const R dz = yz - pz[i];
                    const R r2 = dx * dx + dy * dy + dz * dz;
                    const R ri = MT::rsq(r2);
                    const R r = r2 * ri;
                    // E_m = e^{i k_m r} (masked to 0 for the interior term of
                    // triangles on different objects)
                    R E0r, E0i, E1r, E1i;
                    if constexpr (F32) {
                        MT::template sincos_rev<FR>(r * cf.krev0, E0i, E0r);
                        MT::template sincos_rev<FR>(r * c1.krev1, E1i, E1r);
                    } else {
                        MT::sincos_tab(r * cf.krev0, E0i, E0r, etab);
                        MT::sincos_tab(r * c1.krev1, E1i, E1r, etab);
                    }
                    if (CK0) {
                        const R d0 = MT::exp2(r * cf.kdec0);
                        E0r *= d0;
                        E0i *= d0;
                    }
                    if (CK1 || MULTI) {
                        R d1 = m1;
                        if (CK1) d1 *= MT::exp2(r * c1.kdec1);
                        E1r *= d1;
                        E1i *= d1;
                    }
                    const R G0r = E0r * ri, G0i = E0i * ri;
                    const R G1r = E1r * ri, G1i = E1i * ri;
                    // F r^2 = G_0 (i k_0 r - 1) + G_1 (i k_1 r - 1)
                    //       = i (k_0 E_0 + k_1 E_1) - (G_0 + G_1)       (r / r = 1)
                    R Fr = fmac(c1.ns1, G1r, -G0r), Fi = fmac(c1.ns1, G1i, -G0i);
                    Fr = fmac(-cf.k0r, E0i, Fr);
                    Fi = fmac(cf.k0r, E0r, Fi);
                    Fr = fmac(-c1.k1r, E1i, Fr);
                    Fi = fmac(c1.k1r, E1r, Fi);
                    if (CK0) {
                        Fr = fmac(-cf.k0i, E0r, Fr);
                        Fi = fmac(-cf.k0i, E0i, Fi);
                    }
                    if (CK1) {
                        Fr = fmac(-c1.k1i, E1r, Fr);
                        Fi = fmac(-c1.k1i, E1i, Fi);
                    }
                    const R ri2 = ri * ri;
                    Fr *= ri2;
                    Fi *= ri2;
                    const R GVr = fmac(c1.rho, G1r, G0r), GVi = fmac(c1.rho, G1i, G0i);
                    const R GWr = fmac(c1.irho, G1r, G0r), GWi = fmac(c1.irho, G1i, G0i);
                    // G_0 + (k_1^2 / (rho k_0^2)) G_1
                    R GNr = fmac(c1.n10r, G1r, G0r), GNi = fmac(c1.n10r, G1i, G0i);
                    if (CK0 || CK1) {
                        GNr = fmac(-c1.n10i, G1i, GNr);
                        GNi = fmac(c1.n10i, G1r, GNi);
                    }
                    // complex multiply-accumulates as explicit FMA chains
                    R t1r = a1r[i], t1i = a1i[i], t2r = a2r[i], t2i = a2i[i];
                    t1r = fmac(GVr, spr, t1r);
                    t1r = fmac(-GVi, spi, t1r);
                    t1i = fmac(GVr, spi, t1i);
                    t1i = fmac(GVi, spr, t1i);
                    t2r = fmac(Fr, spxr, t2r);
                    t2r = fmac(-Fi, spxi, t2r);
                    t2i = fmac(Fr, spxi, t2i);
                    t2i = fmac(Fi, spxr, t2i);
                    a1r[i] = t1r;
                    a1i[i] = t1i;
                    a2r[i] = t2r;
                    a2i[i] = t2i;
                    qr[i] = fmac(Fr, sfr, qr[i]);
                    qr[i] = fmac(-Fi, sfi, qr[i]);
                    qi[i] = fmac(Fr, sfi, qi[i]);
                    qi[i] = fmac(Fi, sfr, qi[i]);
                    nr[i] = fmac(GNr, sfr, nr[i]);
                    nr[i] = fmac(-GNi, sfi, nr[i]);
                    ni[i] = fmac(GNr, sfi, ni[i]);
                    ni[i] = fmac(GNi, sfr, ni[i]);
                    const R ww = (R)qw(i) * wj;
                    gwr = fmac(ww, GWr, gwr);
                    gwi = fmac(ww, GWi, gwi);
                }
            }
            // row 1: - F (y - x).n_y s_phi; row 2: - G_N (n_x . n_y) s_phi
            for (int i = 0; i < 6; i++) {
                a1r[i] = fmac(-dny[i], qr[i], a1r[i]);
                a1i[i] = fmac(-dny[i], qi[i], a1i[i]);
                R t2r = a2r[i], t2i = a2i[i];
                t2r = fmac(-gnr, nr[i], t2r);
                t2r = fmac(gni, ni[i], t2r);
                t2i = fmac(-gnr, ni[i], t2i);
                t2i = fmac(-gni, nr[i], t2i);
                a2r[i] = t2r;
                a2i[i] = t2i;
            }
            for (int c = 0; c < 3; c++) {
                const R scr = src[GEO_STRIDE + 24 + 2 * c], sci = src[GEO_STRIDE + 24 + 2 * c + 1];
                Ar[c] += gwr * scr - gwi * sci;
                Ai[c] += gwr * sci + gwi * scr;
            }
        }
        if constexpr (F32) flush();
    }
    flush();
    if (!active) return;
    auto sum_get = [&](int c) -> double {
        if constexpr (F32) return sums[c * nthr + threadIdx.x];
        else return regsum[c];
    };
    double *out = partial + ((int64_t)split * T + tau) * ROW_STRIDE;
    for (int c = 0; c < ROW_STRIDE; c++) out[c] = sum_get(c);
    // the curl accumulator A follows the rows: [nsplit][T][6] after
    // [nsplit][T][12]; the reduction contracts it with the test curls
    double *outA = partial + (int64_t)gridDim.y * T * ROW_STRIDE +
                   ((int64_t)split * T + tau) * 6;
    for (int c = 0; c < 6; c++) outA[c] = sum_get(ROW_STRIDE + c);
}

// ------------------------------------------------- symmetric pair kernel
// G_V, G_W, G_N and F depend on the two points only through r, and the
// geometric factors of K and K' exchange roles when (x, tau) and (y, sigma)
// are swapped: (y_j - x_i).n_sigma = c_sigma - x_i.n_sigma =: dny_i and
// (x_i - y_j).n_tau = c_tau - y_j.n_tau =: dnx_j serve both directions.  So
// every unordered pair of separated triangles tau < sigma is evaluated once
// and its 36 point-pair values feed the rows of tau (test tau, trial sigma)
// and the rows of sigma (test sigma, trial tau), identical sums to the
// one-directional kernel up to the order of additions.
//
// Work item (b, c): the blk test triangles of block b (one per thread)
// against the chunk [b blk + c L, b blk + (c + 1) L) of sigma; pairs with
// tau >= sigma and pairs sharing a vertex are skipped.  Rows of tau: FP32 per
// tile of trial triangles, FP64 sums in LDS, stored at ptau[item][blk][18]
// (12 rows, 6 curl sums).  Rows of sigma: every thread contracts its
// contribution to sigma's three vertices, each wave adds its 64 lanes with a
// fixed DPP tree, the waves' sums are added in FP64 in wave order and stored
// at psig[sig_off(b) - sig_base + sigma - b blk][18].  Every slot is written
// by exactly one work item, so the reduction over slots is deterministic.
// The blocks run in rounds (consecutive block ranges, one launch each) whose
// sigma slots fit a bounded buffer; after each round sym_sig_accum_kernel
// adds its slots to one FP64 sum per sigma, in block order.
constexpr int SIG_VALS = ROW_STRIDE + 6;
constexpr int SYM_WAVES = FF_BLOCK / 64;

// Sum over the 64 lanes of a wave, result in lane 63: quad, row and
// cross-row steps in a fixed order (all lanes must be active).
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_add(float v) {
    const int s = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xF, false);
    return v + __builtin_bit_cast(float, s);
}
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
    v = dpp_add<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v = dpp_add<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    v = dpp_add<0x124, 0xF>(v);   // row_ror:4
    v = dpp_add<0x128, 0xF>(v);   // row_ror:8
    // row broadcasts: rows outside the mask keep v (one masked DPP add; the
    // s_nop covers the two wait states between a VALU write and a DPP read)
    asm volatile("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf"
                 : "+v"(v));
    asm volatile("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf"
                 : "+v"(v));
    return v;
}

// First storage slot of block b in the sigma partials: blocks b' < b hold
// T - b' blk rows each.
__host__ __device__ inline int64_t sym_sig_off(int64_t b, int64_t T, int64_t blk) {
    return b * T - blk * (b * (b - 1) / 2);
}

// Waves per SIMD (measured): 2 for real wavenumbers and one material (256
// VGPRs, nothing spilled: 2.6 % faster than 3), 3 for the lossy and
// several-material variants (their extra exp and table lookups: 5 % faster
// than 2).
template <bool CK0, bool CK1, bool MULTI>
constexpr int sym_waves() { return CK0 || CK1 || MULTI ? 3 : 2; }

template <class R, bool CK0, bool CK1, bool MULTI, bool FR>
__global__ __launch_bounds__(FF_BLOCK) __attribute__((amdgpu_waves_per_eu(sym_waves<CK0, CK1, MULTI>())))
void farfield_sym_kernel(
    const R *__restrict__ geo, const R *__restrict__ dyn,
    const int32_t *__restrict__ tobj, const int32_t *__restrict__ tri, int T,
    const int32_t *__restrict__ items, int chunk_len, Coef<R> cf, const Int<R> *__restrict__ itab,
    double *__restrict__ ptau, double *__restrict__ psig, int64_t sig_base) {
    static_assert(std::is_same<R, float>::value, "symmetric kernel: FP32 only");
    using MT = Math<R>;
    __shared__ R tile[FF_TILE * SRC];
    __shared__ float sig[SYM_WAVES * FF_TILE * SIG_VALS];
    extern __shared__ double sums[];   // [FF_ROWS][blockDim.x]
    const int nthr = blockDim.x;
    const int b = items[3 * blockIdx.x], c = items[3 * blockIdx.x + 1],
              canon = items[3 * blockIdx.x + 2];
    const int tau = b * nthr + threadIdx.x;
    const int lo = b * nthr + c * chunk_len;
    const int hi = min(T, lo + chunk_len);
    const bool active = tau < T;
    const int tt = active ? tau : 0;
    const int wave = threadIdx.x >> 6;
    const bool lane63 = (threadIdx.x & 63) == 63;

    R px[6], py[6], pz[6];
    for (int i = 0; i < 6; i++) {
        px[i] = geo[GEO_STRIDE * tt + 3 * i];
        py[i] = geo[GEO_STRIDE * tt + 3 * i + 1];
        pz[i] = geo[GEO_STRIDE * tt + 3 * i + 2];
    }
    const R ntx = geo[GEO_STRIDE * tt + 18], nty = geo[GEO_STRIDE * tt + 19],
            ntz = geo[GEO_STRIDE * tt + 20], ct = geo[GEO_STRIDE * tt + 21];
    const R ot = MULTI ? (R)tobj[tt] : (R)0;
    const R tv0 = (R)tri[3 * tt], tv1 = (R)tri[3 * tt + 1], tv2 = (R)tri[3 * tt + 2];
    // tau as a trial triangle: s_psi, s_phi at its points, curl sums
    R tspr[6], tspi[6], tsfr[6], tsfi[6], tscr[3], tsci[3];
    for (int i = 0; i < 6; i++) {
        tspr[i] = dyn[DYN_STRIDE * tt + 2 * i];
        tspi[i] = dyn[DYN_STRIDE * tt + 2 * i + 1];
        tsfr[i] = dyn[DYN_STRIDE * tt + 12 + 2 * i];
        tsfi[i] = dyn[DYN_STRIDE * tt + 12 + 2 * i + 1];
    }
    for (int k = 0; k < 3; k++) {
        tscr[k] = dyn[DYN_STRIDE * tt + 24 + 2 * k];
        tsci[k] = dyn[DYN_STRIDE * tt + 24 + 2 * k + 1];
    }

    R a1r[6], a1i[6], a2r[6], a2i[6], Ar[3], Ai[3];
    for (int i = 0; i < 6; i++) a1r[i] = a1i[i] = a2r[i] = a2i[i] = 0;
    for (int k = 0; k < 3; k++) Ar[k] = Ai[k] = 0;
    for (int k = 0; k < FF_ROWS; k++) sums[k * nthr + threadIdx.x] = 0;
    auto flush = [&]() {
        for (int a = 0; a < 3; a++) {
            double r1r = 0, r1i = 0, r2r = 0, r2i = 0;
            for (int i = 0; i < 6; i++) {
                const double wb = qw(i) * qb(i, a);
                r1r += wb * (double)a1r[i];
                r1i += wb * (double)a1i[i];
                r2r += wb * (double)a2r[i];
                r2i += wb * (double)a2i[i];
            }
            sums[(2 * a) * nthr + threadIdx.x] += r1r;
            sums[(2 * a + 1) * nthr + threadIdx.x] += r1i;
            sums[(6 + 2 * a) * nthr + threadIdx.x] += r2r;
            sums[(6 + 2 * a + 1) * nthr + threadIdx.x] += r2i;
        }
        for (int k = 0; k < 3; k++) {
            sums[(ROW_STRIDE + 2 * k) * nthr + threadIdx.x] += (double)Ar[k];
            sums[(ROW_STRIDE + 2 * k + 1) * nthr + threadIdx.x] += (double)Ai[k];
            Ar[k] = Ai[k] = 0;
        }
        for (int i = 0; i < 6; i++) a1r[i] = a1i[i] = a2r[i] = a2i[i] = 0;
    };
    // rows of sigma of one tile: wave sums (LDS) -> FP64 in wave order
    const int nw = nthr >> 6;
    double *psb = psig + (sym_sig_off(b, T, nthr) - sig_base - (int64_t)b * nthr) * SIG_VALS;
    auto combine = [&](int tb, int tcnt) {
        for (int idx = threadIdx.x; idx < tcnt * SIG_VALS; idx += nthr) {
            const int s = idx / SIG_VALS, k = idx - s * SIG_VALS;
            double acc = 0;
            for (int w = 0; w < nw; w++) acc += (double)sig[(w * FF_TILE + s) * SIG_VALS + k];
            psb[(int64_t)(tb + s) * SIG_VALS + k] = acc;
        }
    };

    int prev_base = -1;
    for (int base = lo; base < hi; base += FF_TILE) {
        const int cnt = min(FF_TILE, hi - base);
        __syncthreads();
        if (prev_base >= 0) combine(prev_base, FF_TILE);
        for (int idx = threadIdx.x; idx < cnt * SRC; idx += nthr) {
            int s = idx / SRC, f = idx - s * SRC;
            R v;
            if (f < GEO_STRIDE) v = geo[(int64_t)GEO_STRIDE * (base + s) + f];
            else if (f < GEO_STRIDE + DYN_STRIDE)
                v = dyn[(int64_t)DYN_STRIDE * (base + s) + (f - GEO_STRIDE)];
            else if (f == GEO_STRIDE + DYN_STRIDE) v = MULTI ? (R)tobj[base + s] : (R)0;
            else v = (R)tri[3 * (base + s) + (f - GEO_STRIDE - DYN_STRIDE - 1)];
            tile[idx] = v;
        }
        __syncthreads();
        for (int s = 0; s < cnt; s++) {
            const R *src = &tile[s * SRC];
            const R *sv = src + GEO_STRIDE + DYN_STRIDE + 1;
            const bool adj = sv[0] == tv0 || sv[0] == tv1 || sv[0] == tv2 || sv[1] == tv0 ||
                             sv[1] == tv1 || sv[1] == tv2 || sv[2] == tv0 || sv[2] == tv1 ||
                             sv[2] == tv2;
            // rows of sigma contributed by this thread: 12 rows, 6 curl sums
            R o[SIG_VALS];
            for (int k = 0; k < SIG_VALS; k++) o[k] = 0;
            if (active && tau < base + s && !adj) {
                const R nsx = src[18], nsy = src[19], nsz = src[20], cs = src[21];
                const R m1 = MULTI ? (src[GEO_STRIDE + DYN_STRIDE] == ot ? (R)1 : (R)0) : (R)1;
                const Int<R> c1 = interior<MULTI>(cf, itab, src[GEO_STRIDE + DYN_STRIDE]);
                const R nn = ntx * nsx + nty * nsy + ntz * nsz;
                const R gnr = cf.n0r * nn, gni = cf.n0i * nn;
                // dny_i = (y - x_i).n_sigma; sigma-side trial weights
                // spy_i = dny_i s_psi(x_i)
                R dny[6], spyr[6], spyi[6];
                for (int i = 0; i < 6; i++) {
                    dny[i] = cs - (px[i] * nsx + py[i] * nsy + pz[i] * nsz);
                    spyr[i] = dny[i] * tspr[i];
                    spyi[i] = dny[i] * tspi[i];
                }
                R gwr = 0, gwi = 0;
                // tau at x_i: sums over j of F s_phi(y_j), scaled by dny_i after the loop
                R qtr[6], qti[6];
                for (int i = 0; i < 6; i++) qtr[i] = qti[i] = 0;
                // j stays a loop: the compact body lets two waves issue VALU
                // instructions together more often (measured: 15 % of issue
                // slots instead of 9 %), which outweighs the loop overhead
#pragma unroll 1
                for (int j = 0; j < 6; j++) {
                    // j is the same on every lane: the weight selects stay scalar
                    const int ju = __builtin_amdgcn_readfirstlane(j);
                    const R yx = src[3 * j], yy = src[3 * j + 1], yz = src[3 * j + 2];
                    const R spr = src[GEO_STRIDE + 2 * j], spi = src[GEO_STRIDE + 2 * j + 1];
                    const R sfr = src[GEO_STRIDE + 12 + 2 * j], sfi = src[GEO_STRIDE + 12 + 2 * j + 1];
                    // dnx_j = (x - y_j).n_tau; tau-side weights spx_j = dnx_j s_psi(y_j)
                    // and gsf_j = -k_0^2 (n_x.n_y) s_phi(y_j)
                    const R dnx = ct - (yx * ntx + yy * nty + yz * ntz);
                    const R spxr = dnx * spr, spxi = dnx * spi;
                    const R gsfr = -(gnr * sfr - gni * sfi), gsfi = -(gnr * sfi + gni * sfr);
                    // sigma-side sums over i at y_j
                    R u1r = 0, u1i = 0, qr = 0, qi = 0, u2r = 0, u2i = 0, nr = 0, ni = 0;
#pragma unroll
                    for (int i = 0; i < 6; i++) {
                        const R dx = yx - px[i];
                        const R dy = yy - py[i];
                        const R dz = yz - pz[i];
                        const R r2 = dx * dx + dy * dy + dz * dz;
                        const R ri = MT::rsq(r2);
                        const R r = r2 * ri;
                        R E0r, E0i, E1r, E1i;
                        MT::template sincos_rev<FR>(r * cf.krev0, E0i, E0r);
                        MT::template sincos_rev<FR>(r * c1.krev1, E1i, E1r);
                        if (CK0) {
                            const R d0 = MT::exp2(r * cf.kdec0);
                            E0r *= d0;
                            E0i *= d0;
                        }
                        if (CK1 || MULTI) {
                            R d1 = m1;
                            if (CK1) d1 *= MT::exp2(r * c1.kdec1);
                            E1r *= d1;
                            E1i *= d1;
                        }
                        const R G0r = E0r * ri, G0i = E0i * ri;
                        const R G1r = E1r * ri, G1i = E1i * ri;
                        R Fr = fmac(c1.ns1, G1r, -G0r), Fi = fmac(c1.ns1, G1i, -G0i);
                        Fr = fmac(-cf.k0r, E0i, Fr);
                        Fi = fmac(cf.k0r, E0r, Fi);
                        Fr = fmac(-c1.k1r, E1i, Fr);
                        Fi = fmac(c1.k1r, E1r, Fi);
                        if (CK0) {
                            Fr = fmac(-cf.k0i, E0r, Fr);
                            Fi = fmac(-cf.k0i, E0i, Fi);
                        }
                        if (CK1) {
                            Fr = fmac(-c1.k1i, E1r, Fr);
                            Fi = fmac(-c1.k1i, E1i, Fi);
                        }
                        const R ri2 = ri * ri;
                        Fr *= ri2;
                        Fi *= ri2;
                        const R GVr = fmac(c1.rho, G1r, G0r), GVi = fmac(c1.rho, G1i, G0i);
                        const R GWr = fmac(c1.irho, G1r, G0r), GWi = fmac(c1.irho, G1i, G0i);
                        R GNr = fmac(c1.n10r, G1r, G0r), GNi = fmac(c1.n10r, G1i, G0i);
                        if (CK0 || CK1) {
                            GNr = fmac(-c1.n10i, G1i, GNr);
                            GNi = fmac(c1.n10i, G1r, GNi);
                        }
                        // tau at x_i: G_V s_psi(y_j) - F dny_i s_phi(y_j)
                        //             + F spx_j + G_N gsf_j
                        R t1r = a1r[i], t1i = a1i[i], t2r = a2r[i], t2i = a2i[i];
                        t1r = fmac(GVr, spr, t1r);
                        t1r = fmac(-GVi, spi, t1r);
                        t1i = fmac(GVr, spi, t1i);
                        t1i = fmac(GVi, spr, t1i);
                        qtr[i] = fmac(Fr, sfr, qtr[i]);
                        qtr[i] = fmac(-Fi, sfi, qtr[i]);
                        qti[i] = fmac(Fr, sfi, qti[i]);
                        qti[i] = fmac(Fi, sfr, qti[i]);
                        t2r = fmac(Fr, spxr, t2r);
                        t2r = fmac(-Fi, spxi, t2r);
                        t2i = fmac(Fr, spxi, t2i);
                        t2i = fmac(Fi, spxr, t2i);
                        t2r = fmac(GNr, gsfr, t2r);
                        t2r = fmac(-GNi, gsfi, t2r);
                        t2i = fmac(GNr, gsfi, t2i);
                        t2i = fmac(GNi, gsfr, t2i);
                        a1r[i] = t1r;
                        a1i[i] = t1i;
                        a2r[i] = t2r;
                        a2i[i] = t2i;
                        const R ww = kQW2[6 * ju + i];
                        gwr = fmac(ww, GWr, gwr);
                        gwi = fmac(ww, GWi, gwi);
                        // sigma at y_j: sums over i of G_V s_psi(x_i), F s_phi(x_i),
                        // F spy_i and G_N s_phi(x_i)
                        u1r = fmac(GVr, tspr[i], u1r);
                        u1r = fmac(-GVi, tspi[i], u1r);
                        u1i = fmac(GVr, tspi[i], u1i);
                        u1i = fmac(GVi, tspr[i], u1i);
                        qr = fmac(Fr, tsfr[i], qr);
                        qr = fmac(-Fi, tsfi[i], qr);
                        qi = fmac(Fr, tsfi[i], qi);
                        qi = fmac(Fi, tsfr[i], qi);
                        u2r = fmac(Fr, spyr[i], u2r);
                        u2r = fmac(-Fi, spyi[i], u2r);
                        u2i = fmac(Fr, spyi[i], u2i);
                        u2i = fmac(Fi, spyr[i], u2i);
                        nr = fmac(GNr, tsfr[i], nr);
                        nr = fmac(-GNi, tsfi[i], nr);
                        ni = fmac(GNr, tsfi[i], ni);
                        ni = fmac(GNi, tsfr[i], ni);
                    }
                    // sigma at y_j: row 1 = u1 - dnx_j q; row 2 = u2 - k_0^2 (n.n) n;
                    // contracted with w_j phi_a(y_j)
                    const R r1r = fmac(-dnx, qr, u1r), r1i = fmac(-dnx, qi, u1i);
                    R r2r = fmac(-gnr, nr, u2r), r2i = fmac(-gnr, ni, u2i);
                    r2r = fmac(gni, ni, r2r);
                    r2i = fmac(-gni, nr, r2i);
#pragma unroll
                    for (int a = 0; a < 3; a++) {
                        const R wb = kQWB[3 * ju + a];
                        o[2 * a] = fmac(wb, r1r, o[2 * a]);
                        o[2 * a + 1] = fmac(wb, r1i, o[2 * a + 1]);
                        o[6 + 2 * a] = fmac(wb, r2r, o[6 + 2 * a]);
                        o[6 + 2 * a + 1] = fmac(wb, r2i, o[6 + 2 * a + 1]);
                    }
                }
                for (int i = 0; i < 6; i++) {
                    a1r[i] = fmac(-dny[i], qtr[i], a1r[i]);
                    a1i[i] = fmac(-dny[i], qti[i], a1i[i]);
                }
                // curl terms: A_tau += g_W C_sigma, A_sigma += g_W C_tau
                for (int k = 0; k < 3; k++) {
                    const R scr = src[GEO_STRIDE + 24 + 2 * k], sci = src[GEO_STRIDE + 24 + 2 * k + 1];
                    Ar[k] += gwr * scr - gwi * sci;
                    Ai[k] += gwr * sci + gwi * scr;
                    o[ROW_STRIDE + 2 * k] = gwr * tscr[k] - gwi * tsci[k];
                    o[ROW_STRIDE + 2 * k + 1] = gwr * tsci[k] + gwi * tscr[k];
                }
            }
            float ws[SIG_VALS];
#pragma unroll
            for (int k = 0; k < SIG_VALS; k++) ws[k] = wave_sum_to_lane63((float)o[k]);
            if (lane63) {
#pragma unroll
                for (int k = 0; k < SIG_VALS; k++) sig[(wave * FF_TILE + s) * SIG_VALS + k] = ws[k];
            }
        }
        flush();
        prev_base = base;
    }
    __syncthreads();
    if (prev_base >= 0) combine(prev_base, hi - prev_base);
    if (!active) return;
    double *out = ptau + ((int64_t)canon * nthr + threadIdx.x) * SIG_VALS;
    for (int k = 0; k < SIG_VALS; k++) out[k] = sums[k * nthr + threadIdx.x];
}

// ----------------------------------------- multi-right-hand-side pair kernel
// NR right-hand sides share every kernel evaluation (geometry, phases,
// G_V, G_W, G_N, F); only the accumulations are per right-hand side.  FP32,
// phases below 256 revolutions.  dyn: [NR][T][DYN_STRIDE]; partial of
// right-hand side r at partial + r nsplit T (ROW_STRIDE + 6), same layout
// as the single-vector kernel.  Per-tile FP64 sums are accumulated in place
// in the thread's own partial slots.
template <int NR> constexpr int srcm() { return GEO_STRIDE + 4 + NR * DYN_STRIDE; }

template <class R, int NR> constexpr int multi_waves() {
    return std::is_same<R, double>::value || NR >= 4 ? 1 : 2;
}

template <class R, bool CK0, bool CK1, bool MULTI, int NR>
__global__ __launch_bounds__(FF_BLOCK) __attribute__((amdgpu_waves_per_eu(multi_waves<R, NR>())))
void farfield_multi_kernel(
    const R *__restrict__ geo, const R *__restrict__ dyn,
    const int32_t *__restrict__ tobj, const int32_t *__restrict__ tri, int T,
    int split_len, Coef<R> cf, const Int<R> *__restrict__ itab,
    double *__restrict__ partial) {
    using MT = Math<R>;
    // FP32 phases are below 256 revolutions on this path; FP64 always reduces
    constexpr bool FRM = std::is_same<R, double>::value;
    constexpr int SM = srcm<NR>();
    constexpr int OBJ = GEO_STRIDE, VID = GEO_STRIDE + 1, DYN0 = GEO_STRIDE + 4;
    __shared__ R tile[FF_TILE * SM];
    __shared__ double2 etab[FRM ? 256 : 1];
    const int nthr = blockDim.x;
    const int tau = blockIdx.x * nthr + threadIdx.x;
    if constexpr (FRM) {
        for (int n = threadIdx.x; n < 256; n += nthr) {
            double sn, cs;
            MT::template sincos_rev<true>(n * 0.00390625, sn, cs);
            etab[n] = make_double2(cs, sn);
        }
        // the first tile's barrier orders these writes before any read
    }
    const int split = blockIdx.y;
    const int s_begin = split * split_len;
    const int s_end = min(T, s_begin + split_len);
    const bool active = tau < T;
    const int tt = active ? tau : 0;

    R px[6], py[6], pz[6];
    for (int i = 0; i < 6; i++) {
        px[i] = geo[GEO_STRIDE * tt + 3 * i];
        py[i] = geo[GEO_STRIDE * tt + 3 * i + 1];
        pz[i] = geo[GEO_STRIDE * tt + 3 * i + 2];
    }
    const R ntx = geo[GEO_STRIDE * tt + 18], nty = geo[GEO_STRIDE * tt + 19],
            ntz = geo[GEO_STRIDE * tt + 20], ct = geo[GEO_STRIDE * tt + 21];
    const R ot = MULTI ? (R)tobj[tt] : (R)0;
    const R tv0 = (R)tri[3 * tt], tv1 = (R)tri[3 * tt + 1], tv2 = (R)tri[3 * tt + 2];

    R a1r[NR][6], a1i[NR][6], a2r[NR][6], a2i[NR][6], Ar[NR][3], Ai[NR][3];
    for (int r = 0; r < NR; r++) {
        for (int i = 0; i < 6; i++) a1r[r][i] = a1i[r][i] = a2r[r][i] = a2i[r][i] = 0;
        for (int c = 0; c < 3; c++) Ar[r][c] = Ai[r][c] = 0;
    }
    const int64_t rstride = (int64_t)gridDim.y * T * (ROW_STRIDE + 6);
    double *out = partial + ((int64_t)split * T + tau) * ROW_STRIDE;
    double *outA = partial + (int64_t)gridDim.y * T * ROW_STRIDE + ((int64_t)split * T + tau) * 6;
    bool first = true;
    auto flush = [&]() {
        for (int r = 0; r < NR; r++) {
            double v[ROW_STRIDE + 6];
            for (int a = 0; a < 3; a++) {
                double r1r = 0, r1i = 0, r2r = 0, r2i = 0;
                for (int i = 0; i < 6; i++) {
                    double wb = qw(i) * qb(i, a);
                    r1r += wb * (double)a1r[r][i];
                    r1i += wb * (double)a1i[r][i];
                    r2r += wb * (double)a2r[r][i];
                    r2i += wb * (double)a2i[r][i];
                }
                v[2 * a] = r1r;
                v[2 * a + 1] = r1i;
                v[6 + 2 * a] = r2r;
                v[6 + 2 * a + 1] = r2i;
            }
            for (int c = 0; c < 3; c++) {
                v[ROW_STRIDE + 2 * c] = (double)Ar[r][c];
                v[ROW_STRIDE + 2 * c + 1] = (double)Ai[r][c];
                Ar[r][c] = Ai[r][c] = 0;
            }
            for (int i = 0; i < 6; i++) a1r[r][i] = a1i[r][i] = a2r[r][i] = a2i[r][i] = 0;
            if (active) {
                double *o = out + r * rstride, *oA = outA + r * rstride;
                for (int c = 0; c < ROW_STRIDE; c++) o[c] = first ? v[c] : o[c] + v[c];
                for (int c = 0; c < 6; c++) oA[c] = first ? v[ROW_STRIDE + c] : oA[c] + v[ROW_STRIDE + c];
            }
        }
        first = false;
    };

    for (int base = s_begin; base < s_end; base += FF_TILE) {
        const int cnt = min(FF_TILE, s_end - base);
        __syncthreads();
        for (int idx = threadIdx.x; idx < cnt * SM; idx += nthr) {
            const int sl = idx / SM, f = idx - sl * SM;
            R v;
            if (f < GEO_STRIDE) v = geo[(int64_t)GEO_STRIDE * (base + sl) + f];
            else if (f == OBJ) v = MULTI ? (R)tobj[base + sl] : (R)0;
            else if (f < DYN0) v = (R)tri[3 * (base + sl) + (f - VID)];
            else {
                const int r = (f - DYN0) / DYN_STRIDE, c = f - DYN0 - r * DYN_STRIDE;
                v = dyn[((int64_t)r * T + base + sl) * DYN_STRIDE + c];
            }
            tile[idx] = v;
        }
        __syncthreads();
        for (int sl = 0; sl < cnt; sl++) {
            const R *src = &tile[sl * SM];
            {
                const R *sv = src + VID;
                const bool adj = sv[0] == tv0 || sv[0] == tv1 || sv[0] == tv2 ||
                                 sv[1] == tv0 || sv[1] == tv1 || sv[1] == tv2 ||
                                 sv[2] == tv0 || sv[2] == tv1 || sv[2] == tv2;
                if (adj) continue;   // includes sigma == tau: near field
            }
            const R nsx = src[18], nsy = src[19], nsz = src[20], cs = src[21];
            const R m1 = MULTI ? (src[OBJ] == ot ? (R)1 : (R)0) : (R)1;
            const Int<R> c1 = interior<MULTI>(cf, itab, src[OBJ]);
            const R nn = ntx * nsx + nty * nsy + ntz * nsz;
            const R gnr = cf.n0r * nn, gni = cf.n0i * nn;
            R dnx[6], dny[6];
            for (int j = 0; j < 6; j++)
                dnx[j] = ct - (src[3 * j] * ntx + src[3 * j + 1] * nty + src[3 * j + 2] * ntz);
            for (int i = 0; i < 6; i++)
                dny[i] = cs - (px[i] * nsx + py[i] * nsy + pz[i] * nsz);
            R gwr = 0, gwi = 0;
#pragma unroll
            for (int i = 0; i < 6; i++) {
                R qr[NR], qi[NR], nr[NR], ni[NR];
                for (int r = 0; r < NR; r++) qr[r] = qi[r] = nr[r] = ni[r] = 0;
#pragma unroll
                for (int j = 0; j < 6; j++) {
                    const R dx = src[3 * j] - px[i];
                    const R dy = src[3 * j + 1] - py[i];
                    const R dz = src[3 * j + 2] - pz[i];
                    const R r2 = dx * dx + dy * dy + dz * dz;
                    const R ri = MT::rsq(r2);
                    const R rr = r2 * ri;
                    R E0r, E0i, E1r, E1i;
                    if constexpr (FRM) {
                        MT::sincos_tab(rr * cf.krev0, E0i, E0r, etab);
                        MT::sincos_tab(rr * c1.krev1, E1i, E1r, etab);
                    } else {
                        MT::template sincos_rev<false>(rr * cf.krev0, E0i, E0r);
                        MT::template sincos_rev<false>(rr * c1.krev1, E1i, E1r);
                    }
                    if (CK0) {
                        const R d0 = MT::exp2(rr * cf.kdec0);
                        E0r *= d0;
                        E0i *= d0;
                    }
                    if (CK1 || MULTI) {
                        R d1 = m1;
                        if (CK1) d1 *= MT::exp2(rr * c1.kdec1);
                        E1r *= d1;
                        E1i *= d1;
                    }
                    const R G0r = E0r * ri, G0i = E0i * ri;
                    const R G1r = E1r * ri, G1i = E1i * ri;
                    R Fr = fmac(c1.ns1, G1r, -G0r), Fi = fmac(c1.ns1, G1i, -G0i);
                    Fr = fmac(-cf.k0r, E0i, Fr);
                    Fi = fmac(cf.k0r, E0r, Fi);
                    Fr = fmac(-c1.k1r, E1i, Fr);
                    Fi = fmac(c1.k1r, E1r, Fi);
                    if (CK0) {
                        Fr = fmac(-cf.k0i, E0r, Fr);
                        Fi = fmac(-cf.k0i, E0i, Fi);
                    }
                    if (CK1) {
                        Fr = fmac(-c1.k1i, E1r, Fr);
                        Fi = fmac(-c1.k1i, E1i, Fi);
                    }
                    const R ri2 = ri * ri;
                    Fr *= ri2;
                    Fi *= ri2;
                    const R GVr = fmac(c1.rho, G1r, G0r), GVi = fmac(c1.rho, G1i, G0i);
                    const R GWr = fmac(c1.irho, G1r, G0r), GWi = fmac(c1.irho, G1i, G0i);
                    R GNr = fmac(c1.n10r, G1r, G0r), GNi = fmac(c1.n10r, G1i, G0i);
                    if (CK0 || CK1) {
                        GNr = fmac(-c1.n10i, G1i, GNr);
                        GNi = fmac(c1.n10i, G1r, GNi);
                    }
                    const R Fxr = Fr * dnx[j], Fxi = Fi * dnx[j];
#pragma unroll
                    for (int r = 0; r < NR; r++) {
                        const R *d = src + DYN0 + r * DYN_STRIDE;
                        const R spr = d[2 * j], spi = d[2 * j + 1];
                        const R sfr = d[12 + 2 * j], sfi = d[12 + 2 * j + 1];
                        R t1r = a1r[r][i], t1i = a1i[r][i], t2r = a2r[r][i], t2i = a2i[r][i];
                        t1r = fmac(GVr, spr, t1r);
                        t1r = fmac(-GVi, spi, t1r);
                        t1i = fmac(GVr, spi, t1i);
                        t1i = fmac(GVi, spr, t1i);
                        qr[r] = fmac(Fr, sfr, qr[r]);
                        qr[r] = fmac(-Fi, sfi, qr[r]);
                        qi[r] = fmac(Fr, sfi, qi[r]);
                        qi[r] = fmac(Fi, sfr, qi[r]);
                        t2r = fmac(Fxr, spr, t2r);
                        t2r = fmac(-Fxi, spi, t2r);
                        t2i = fmac(Fxr, spi, t2i);
                        t2i = fmac(Fxi, spr, t2i);
                        nr[r] = fmac(GNr, sfr, nr[r]);
                        nr[r] = fmac(-GNi, sfi, nr[r]);
                        ni[r] = fmac(GNr, sfi, ni[r]);
                        ni[r] = fmac(GNi, sfr, ni[r]);
                        a1r[r][i] = t1r;
                        a1i[r][i] = t1i;
                        a2r[r][i] = t2r;
                        a2i[r][i] = t2i;
                    }
                    const R ww = (R)(qw(i) * qw(j));
                    gwr = fmac(ww, GWr, gwr);
                    gwi = fmac(ww, GWi, gwi);
                }
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    a1r[r][i] = fmac(-dny[i], qr[r], a1r[r][i]);
                    a1i[r][i] = fmac(-dny[i], qi[r], a1i[r][i]);
                    R t2r = a2r[r][i], t2i = a2i[r][i];
                    t2r = fmac(-gnr, nr[r], t2r);
                    t2r = fmac(gni, ni[r], t2r);
                    t2i = fmac(-gnr, ni[r], t2i);
                    t2i = fmac(-gni, nr[r], t2i);
                    a2r[r][i] = t2r;
                    a2i[r][i] = t2i;
                }
            }
#pragma unroll
            for (int r = 0; r < NR; r++) {
                const R *d = src + DYN0 + r * DYN_STRIDE;
                for (int c = 0; c < 3; c++) {
                    const R scr = d[24 + 2 * c], sci = d[24 + 2 * c + 1];
                    Ar[r][c] += gwr * scr - gwi * sci;
                    Ai[r][c] += gwr * sci + gwi * scr;
                }
            }
        }
        flush();
    }
    if (first) flush();   // empty split: zero partials
}

// --------------------------------------------------------- split reduction
// trirows[tau][c] = |tau|/(4 pi) * sum_split (rows + curl term), fixed order.
__global__ __launch_bounds__(256) void reduce_splits_kernel(
    const double *__restrict__ partial, const double *__restrict__ tst, int T,
    int nsplit, double *__restrict__ trirows) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double acc[12], A[6];
    for (int c = 0; c < 12; c++) acc[c] = 0;
    for (int c = 0; c < 6; c++) A[c] = 0;
    const double *pa = partial + (int64_t)nsplit * T * ROW_STRIDE;
    for (int s = 0; s < nsplit; s++) {
        const double *p = partial + ((int64_t)s * T + t) * ROW_STRIDE;
        for (int c = 0; c < 12; c++) acc[c] += p[c];
        const double *q = pa + ((int64_t)s * T + t) * 6;
        for (int c = 0; c < 6; c++) A[c] += q[c];
    }
    const double *ts = tst + (int64_t)TST_STRIDE * t;
    const double sc = ts[0] * 0.079577471545947667884441881686257;   // |tau|/(4 pi)
    for (int a = 0; a < 3; a++) {
        const double *cu = ts + 1 + 3 * a;
        acc[6 + 2 * a] += cu[0] * A[0] + cu[1] * A[2] + cu[2] * A[4];
        acc[6 + 2 * a + 1] += cu[0] * A[1] + cu[1] * A[3] + cu[2] * A[5];
    }
    for (int c = 0; c < 12; c++) trirows[(int64_t)ROW_STRIDE * t + c] = sc * acc[c];
}

// ------------------------------------------- symmetric-kernel reduction
// Rows of test triangle tau from the symmetric kernel: its own work items
// as tau (chunk order), then its sum as sigma over the blocks b <=
// block(tau); then the curl contraction and |tau|/(4 pi) as in the split
// reduction.
// sigacc[sigma] (+)= the slots of blocks [b0, b1) for sigma (block order;
// the round of block 0 starts every sum)
__global__ __launch_bounds__(256) void sym_sig_accum_kernel(
    const double *__restrict__ psig, int64_t sig_base, int b0, int b1, int T, int blk,
    double *__restrict__ sigacc) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T || t < b0 * blk) return;
    double acc[SIG_VALS];
    double *o = sigacc + (int64_t)t * SIG_VALS;
    for (int k = 0; k < SIG_VALS; k++) acc[k] = b0 == 0 ? 0.0 : o[k];
    const int last = min(b1 - 1, t / blk);
    for (int bb = b0; bb <= last; bb++) {
        const double *q = psig + (sym_sig_off(bb, T, blk) - sig_base + t - (int64_t)bb * blk) * SIG_VALS;
        for (int k = 0; k < SIG_VALS; k++) acc[k] += q[k];
    }
    for (int k = 0; k < SIG_VALS; k++) o[k] = acc[k];
}

__global__ __launch_bounds__(256) void reduce_sym_kernel(
    const double *__restrict__ ptau, const double *__restrict__ sigacc,
    const double *__restrict__ tst, int T, int blk, int chunk_len,
    double *__restrict__ trirows) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const int b = t / blk, l = t - b * blk;
    int64_t first = 0;
    for (int bb = 0; bb < b; bb++) first += (T - bb * blk + chunk_len - 1) / chunk_len;
    const int nch = (T - b * blk + chunk_len - 1) / chunk_len;
    double acc[SIG_VALS];
    for (int k = 0; k < SIG_VALS; k++) acc[k] = 0;
    for (int c = 0; c < nch; c++) {
        const double *p = ptau + ((first + c) * blk + l) * SIG_VALS;
        for (int k = 0; k < SIG_VALS; k++) acc[k] += p[k];
    }
    {
        const double *q = sigacc + (int64_t)t * SIG_VALS;
        for (int k = 0; k < SIG_VALS; k++) acc[k] += q[k];
    }
    const double *ts = tst + (int64_t)TST_STRIDE * t;
    const double sc = ts[0] * 0.079577471545947667884441881686257;   // |tau|/(4 pi)
    const double *A = acc + ROW_STRIDE;
    for (int a = 0; a < 3; a++) {
        const double *cu = ts + 1 + 3 * a;
        acc[6 + 2 * a] += cu[0] * A[0] + cu[1] * A[2] + cu[2] * A[4];
        acc[6 + 2 * a + 1] += cu[0] * A[1] + cu[1] * A[3] + cu[2] * A[5];
    }
    for (int c = 0; c < ROW_STRIDE; c++) trirows[(int64_t)ROW_STRIDE * t + c] = sc * acc[c];
}

// ------------------------------------- vertex gather + near-field CSR SpMV
__global__ __launch_bounds__(256) void finalize_kernel(
    const double *__restrict__ trirows, const int32_t *__restrict__ star_ptr,
    const int32_t *__restrict__ star_idx, const int32_t *__restrict__ rowptr,
    const int32_t *__restrict__ col, const double2 *__restrict__ nf, int64_t nnz,
    const double2 *__restrict__ x, int64_t N, double2 *__restrict__ y) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double y1r = 0, y1i = 0, y2r = 0, y2i = 0;
    for (int e = star_ptr[i]; e < star_ptr[i + 1]; e++) {
        int ta = star_idx[e];
        int t = ta / 3, a = ta - 3 * t;
        const double *r = trirows + (int64_t)ROW_STRIDE * t;
        y1r += r[2 * a];
        y1i += r[2 * a + 1];
        y2r += r[6 + 2 * a];
        y2i += r[6 + 2 * a + 1];
    }
    const double2 *C11 = nf, *C12 = nf + nnz, *C21 = nf + 2 * nnz, *C22 = nf + 3 * nnz;
    for (int e = rowptr[i]; e < rowptr[i + 1]; e++) {
        int j = col[e];
        double2 p = x[j], f = x[N + j];
        double2 a = C11[e], b = C12[e], c = C21[e], d = C22[e];
        y1r += a.x * p.x - a.y * p.y + b.x * f.x - b.y * f.y;
        y1i += a.x * p.y + a.y * p.x + b.x * f.y + b.y * f.x;
        y2r += c.x * p.x - c.y * p.y + d.x * f.x - d.y * f.y;
        y2i += c.x * p.y + c.y * p.x + d.x * f.y + d.y * f.x;
    }
    y[i] = make_double2(y1r, y1i);
    y[N + i] = make_double2(y2r, y2i);
}

// s1 = +1: PMCHWT (A_0 + A^_1); s1 = -1: the interior terms of the Mueller
// operator (A_0 - A^_1).  The sign is folded into every interior coefficient:
// rho, 1/rho, k_1^2/(rho k_0^2) and k_1 (which enters only through F), and
// ns1 carries it into the -(G_0 + s1 G_1) part of F.
template <class R> Int<R> make_int(double2 k0, double2 k1, double rho, int s1) {
    Int<R> c;
    const double inv2pi = 0.15915494309189533576888376337251;
    const double log2e = 1.4426950408889634073599246810019;
    c.krev1 = (R)(k1.x * inv2pi);
    c.k1r = (R)k1.x;
    c.k1i = (R)k1.y;
    c.kdec1 = (R)(-k1.y * log2e);
    c.rho = (R)rho;
    c.irho = (R)(1.0 / rho);
    // k_1^2 / (rho k_0^2); k_0 != 0 is checked at the entry points
    const double n0r = k0.x * k0.x - k0.y * k0.y, n0i = 2.0 * k0.x * k0.y;
    const double n1r = (k1.x * k1.x - k1.y * k1.y) / rho, n1i = 2.0 * k1.x * k1.y / rho;
    const double d = n0r * n0r + n0i * n0i;
    c.n10r = (R)((n1r * n0r + n1i * n0i) / d);
    c.n10i = (R)((n1i * n0r - n1r * n0i) / d);
    if (s1 < 0) {
        c.k1r = -c.k1r;
        c.k1i = -c.k1i;
        c.rho = -c.rho;
        c.irho = -c.irho;
        c.n10r = -c.n10r;
        c.n10i = -c.n10i;
    }
    c.ns1 = (R)(s1 < 0 ? 1.0 : -1.0);
    return c;
}

// Launch coefficients from the near-field operator's materials: the first
// object's interior part by value (one object); kernels for several objects
// read every object's from interior_table().
template <class R> Coef<R> make_coef(double2 k0, const NearOperator &nf) {
    Coef<R> c;
    const double inv2pi = 0.15915494309189533576888376337251;
    const double log2e = 1.4426950408889634073599246810019;
    c.krev0 = (R)(k0.x * inv2pi);
    c.k0r = (R)k0.x;
    c.k0i = (R)k0.y;
    c.kdec0 = (R)(-k0.y * log2e);
    c.n0r = (R)(k0.x * k0.x - k0.y * k0.y);
    c.n0i = (R)(2.0 * k0.x * k0.y);
    c.in = make_int<R>(k0, nf.k1o[0], nf.rhoo[0], nf.s1);
    return c;
}

// per-object interior coefficients on the device (built on first use, kept
// with the near-field operator), or nullptr for one object
template <class R> const Int<R> *interior_table(const bem_mesh *m, const NearOperator &nf,
                                                double2 k0) {
    if (m->nobj < 2) return nullptr;
    static_assert(sizeof(Int<R>) == INT_COEFS * sizeof(R), "Int<R> layout");
    constexpr bool F32 = std::is_same<R, float>::value;
    auto &buf = [&]() -> auto & {
        if constexpr (F32) return nf.itab32;
        else return nf.itab64;
    }();
    if (!buf.p) {
        std::vector<R> h((size_t)m->nobj * INT_COEFS);
        for (int o = 0; o < m->nobj; o++) {
            const Int<R> c = make_int<R>(k0, nf.k1o[o], nf.rhoo[o], nf.s1);
            std::memcpy(h.data() + (size_t)o * INT_COEFS, &c, sizeof(c));
        }
        buf.upload(h);
    }
    return (const Int<R> *)buf.p;
}

// dynamic LDS of the single-vector kernel: FP32 per-thread FP64 sums
template <class R> size_t far_smem(int blk) {
    return std::is_same<R, float>::value ? (size_t)FF_ROWS * blk * sizeof(double) : 0;
}

template <class R, bool CK0, bool CK1, bool MULTI, bool FR>
void launch_far(dim3 grid, int blk, hipStream_t s, const R *geo, const R *dyn,
                const int32_t *tobj, const int32_t *tri, int T, int split_len, Coef<R> cf,
                const Int<R> *itab, double *partial) {
    hipLaunchKernelGGL((farfield_kernel<R, CK0, CK1, MULTI, FR>), grid, dim3(blk), far_smem<R>(blk),
                       s, geo, dyn, tobj, tri, T, split_len, cf, itab, partial);
}

// fr: reduce phases to [0, 1) revolutions before v_sin/v_cos (needed when
// k r / 2 pi can reach 256); the FP64 path always reduces.
template <class R, bool FR>
void dispatch_far(dim3 grid, int blk, hipStream_t s, const R *geo, const R *dyn,
                  const int32_t *tobj, const int32_t *tri, int T, int split_len, Coef<R> cf,
                  const Int<R> *itab, double *partial, bool ck0, bool ck1, bool multi) {
    int code = (ck0 ? 4 : 0) | (ck1 ? 2 : 0) | (multi ? 1 : 0);
    switch (code) {
#define BEM_CASE(c, a, b, m) \
    case c:                                                                                      \
        launch_far<R, a, b, m, FR>(grid, blk, s, geo, dyn, tobj, tri, T, split_len, cf, itab,    \
                                   partial);                                                     \
        break;
        BEM_CASE(0, false, false, false)
        BEM_CASE(1, false, false, true)
        BEM_CASE(2, false, true, false)
        BEM_CASE(3, false, true, true)
        BEM_CASE(4, true, false, false)
        BEM_CASE(5, true, false, true)
        BEM_CASE(6, true, true, false)
        BEM_CASE(7, true, true, true)
#undef BEM_CASE
    }
}

// Pair kernel variant for the runtime flags (code = 4 ck0 + 2 ck1 + multi).
template <class R, bool FR> const void *far_kernel(int code) {
    switch (code) {
    case 0: return (const void *)farfield_kernel<R, false, false, false, FR>;
    case 1: return (const void *)farfield_kernel<R, false, false, true, FR>;
    case 2: return (const void *)farfield_kernel<R, false, true, false, FR>;
    case 3: return (const void *)farfield_kernel<R, false, true, true, FR>;
    case 4: return (const void *)farfield_kernel<R, true, false, false, FR>;
    case 5: return (const void *)farfield_kernel<R, true, false, true, FR>;
    case 6: return (const void *)farfield_kernel<R, true, true, false, FR>;
    default: return (const void *)farfield_kernel<R, true, true, true, FR>;
    }
}

template <class R, int NR> const void *multi_kernel(int code) {
    switch (code) {
    case 0: return (const void *)farfield_multi_kernel<R, false, false, false, NR>;
    case 1: return (const void *)farfield_multi_kernel<R, false, false, true, NR>;
    case 2: return (const void *)farfield_multi_kernel<R, false, true, false, NR>;
    case 3: return (const void *)farfield_multi_kernel<R, false, true, true, NR>;
    case 4: return (const void *)farfield_multi_kernel<R, true, false, false, NR>;
    case 5: return (const void *)farfield_multi_kernel<R, true, false, true, NR>;
    case 6: return (const void *)farfield_multi_kernel<R, true, true, false, NR>;
    default: return (const void *)farfield_multi_kernel<R, true, true, true, NR>;
    }
}

template <class R, int NR>
void launch_multi(int code, dim3 grid, int blk, hipStream_t s, const R *geo, const R *dyn,
                  const int32_t *tobj, const int32_t *tri, int T, int split_len, Coef<R> cf,
                  const Int<R> *itab, double *partial) {
    switch (code) {
#define BEM_CASE(c, a, b, m)                                                                     \
    case c:                                                                                      \
        hipLaunchKernelGGL((farfield_multi_kernel<R, a, b, m, NR>), grid, dim3(blk), 0, s,      \
                           geo, dyn, tobj, tri, T, split_len, cf, itab, partial);                \
        break;
        BEM_CASE(0, false, false, false)
        BEM_CASE(1, false, false, true)
        BEM_CASE(2, false, true, false)
        BEM_CASE(3, false, true, true)
        BEM_CASE(4, true, false, false)
        BEM_CASE(5, true, false, true)
        BEM_CASE(6, true, true, false)
        BEM_CASE(7, true, true, true)
#undef BEM_CASE
    }
}

// Workgroups of a pair kernel variant resident on the current device at once
// (compute units x occupancy) for a block size and dynamic LDS, cached per
// device and variant.
int far_slots(const void *kern, int blk, size_t smem) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void *, int>, int> cache;
    int dev = 0;
    BEM_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find({dev, kern, blk});
    if (it != cache.end()) return it->second;
    int cus = 0, per_cu = 0;
    BEM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    BEM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, blk, smem));
    const int slots = std::max(1, cus * per_cu);
    cache[{dev, kern, blk}] = slots;
    return slots;
}

}   // namespace

// Number of trial-triangle splits (grid.y).  Every workgroup of a launch costs
// about the same, so the launch runs in rounds of `slots` resident
// workgroups; the split count minimises rounds x (trial triangles per split
// + a small fixed cost), which avoids a nearly empty last round.
int farfield_splits(int T, int slots, int blk) {
    const int tiles = (T + blk - 1) / blk;
    const int max_s = std::max(1, (T + FF_TILE - 1) / FF_TILE);
    const double fixed = 2.0;   // prologue + flush, in trial triangles
    int best = 1;
    double best_cost = 1e300;
    for (int sp = 1; sp <= max_s; sp++) {
        const int len = (T + sp - 1) / sp;
        const long long rounds = ((long long)tiles * sp + slots - 1) / slots;
        const double cost = (double)rounds * (len + fixed);
        if (cost < best_cost * (1.0 - 1e-12)) {
            best_cost = cost;
            best = sp;
        }
    }
    return best;
}

namespace {

// Launch plan of the pair kernel for one precision and wavenumber pair.
struct FarPlan {
    int code;      // 4 ck0 + 2 ck1 + multi
    bool fr;       // phase reduction before v_sin/v_cos (FP32)
    int blk;       // test triangles per workgroup
    int nsplit;    // trial-triangle splits (grid.y)
};

FarPlan far_plan(const bem_mesh *m, int precision, double2 k0, double2 k1, int blk) {
    FarPlan p;
    const bool ck0 = k0.y != 0.0, ck1 = k1.y != 0.0, multi = m->nobj > 1;
    p.code = (ck0 ? 4 : 0) | (ck1 ? 2 : 0) | (multi ? 1 : 0);
    // largest phase in revolutions: max Re k * diameter / (2 pi)
    const double tmax = std::max(std::fabs(k0.x), std::fabs(k1.x)) * m->diameter *
                        0.15915494309189533576888376337251;
    p.fr = precision != BEM_FP32 || tmax >= 256.0;
    p.blk = blk;
    const void *kern = precision == BEM_FP32
                           ? (p.fr ? far_kernel<float, true>(p.code)
                                   : far_kernel<float, false>(p.code))
                           : far_kernel<double, true>(p.code);
    const size_t smem = precision == BEM_FP32 ? far_smem<float>(blk) : 0;
    p.nsplit = farfield_splits((int)m->T, far_slots(kern, blk, smem), blk);
    return p;
}

int valid_block(int b) { return b == 64 || b == 128 || b == 256 ? b : 256; }

// Symmetric kernel variant for the runtime flags (code = 4 ck0 + 2 ck1 + multi).
template <bool FR> const void *sym_kernel(int code) {
    switch (code) {
    case 0: return (const void *)farfield_sym_kernel<float, false, false, false, FR>;
    case 1: return (const void *)farfield_sym_kernel<float, false, false, true, FR>;
    case 2: return (const void *)farfield_sym_kernel<float, false, true, false, FR>;
    case 3: return (const void *)farfield_sym_kernel<float, false, true, true, FR>;
    case 4: return (const void *)farfield_sym_kernel<float, true, false, false, FR>;
    case 5: return (const void *)farfield_sym_kernel<float, true, false, true, FR>;
    case 6: return (const void *)farfield_sym_kernel<float, true, true, false, FR>;
    default: return (const void *)farfield_sym_kernel<float, true, true, true, FR>;
    }
}

template <bool FR>
void launch_sym(int code, int n_items, int blk, hipStream_t s, const float *geo, const float *dyn,
                const int32_t *tobj, const int32_t *tri, int T, const int32_t *items, int chunk,
                Coef<float> cf, const Int<float> *itab, double *ptau, double *psig,
                int64_t sig_base) {
    switch (code) {
#define BEM_CASE(c, a, b, m)                                                                     \
    case c:                                                                                      \
        hipLaunchKernelGGL((farfield_sym_kernel<float, a, b, m, FR>), dim3(n_items), dim3(blk),  \
                           far_smem<float>(blk), s, geo, dyn, tobj, tri, T, items, chunk, cf,    \
                           itab, ptau, psig, sig_base);                                          \
        break;
        BEM_CASE(0, false, false, false)
        BEM_CASE(1, false, false, true)
        BEM_CASE(2, false, true, false)
        BEM_CASE(3, false, true, true)
        BEM_CASE(4, true, false, false)
        BEM_CASE(5, true, false, true)
        BEM_CASE(6, true, true, false)
        BEM_CASE(7, true, true, true)
#undef BEM_CASE
    }
}

// Work items of the symmetric kernel.  Block b (test triangles
// [b blk, b blk + blk)) meets the trial triangles [b blk, T) in chunks of
// `chunk`; the chunk length is the multiple of the tile that minimises the
// makespan of a greedy list schedule of the items (longest first) on the
// resident workgroup slots, among lengths giving 1.5 to 8 items per slot.  Launch order: full chunks, then the shorter
// last chunks by decreasing length; storage order of the tau rows: b-major.
// Rounds: consecutive block ranges [b0, b1) whose sigma slots take at most
// "farfield.sym_round_mib" (one launch each), their items at [item0, item0 +
// nitems).
struct SymRound {
    int b0, b1, item0, nitems;
    int64_t sig_base;   // sym_sig_off(b0)
};
struct SymPlan {
    int blk = 0, chunk = 0, nblk = 0;
    std::vector<int32_t> items;   // launch order, round after round: (b, c, storage index)
    std::vector<SymRound> rounds;
    int64_t tau_doubles = 0, sig_doubles = 0;   // sig_doubles: the largest round
};

const SymPlan &sym_plan(int T, int blk, int slots) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int>, SymPlan> cache;
    const int cap_mib = tuning().farfield_sym_round_mib.load();
    const int64_t sig_cap = (int64_t)cap_mib << 20;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find({T, blk, slots, cap_mib});
    if (it != cache.end()) return it->second;
    const int nblk = (T + blk - 1) / blk;
    // rounds: consecutive blocks whose sigma slots fit the cap
    std::vector<std::pair<int, int>> rounds;
    for (int b0 = 0; b0 < nblk;) {
        int b1 = b0 + 1;
        while (b1 < nblk && (sym_sig_off(b1 + 1, T, blk) - sym_sig_off(b0, T, blk)) * SIG_VALS *
                                    (int64_t)sizeof(double) <= sig_cap)
            b1++;
        rounds.emplace_back(b0, b1);
        b0 = b1;
    }
    const int64_t nr = (int64_t)rounds.size();
    const double fixed = 2.0;
    int best_L = T;
    double best_cost = 1e300;
    std::vector<int> lens;
    // At about one item per slot the launch measured 8 % slower than the
    // schedule predicts (icosphere L5: 17.2 ms at 800 items, 15.9 ms at 1562
    // on 768 slots), so lengths giving at least 1.5 items per slot and round
    // are preferred where the mesh has enough pairs; each round is a launch
    // of its own, so the cost is the sum of the rounds' makespans.
    int64_t max_items = 0;
    for (int b = 0; b < nblk; b++) max_items += (T - b * blk + FF_TILE - 1) / FF_TILE;
    const int64_t min_items = std::min<int64_t>(3 * (int64_t)slots / 2 * nr, max_items);
    for (int L = FF_TILE; L < T + FF_TILE; L += FF_TILE) {
        int64_t n_items = 0;
        for (int b = 0; b < nblk; b++) n_items += (T - b * blk + L - 1) / L;
        // beyond a few rounds finer chunks only add partial-buffer traffic
        if (n_items > std::min<int64_t>(50000, 8 * (int64_t)slots * nr)) continue;
        if (n_items < min_items) break;   // fewer items for every longer chunk
        double cost = 0;
        for (const auto &r : rounds) {
            lens.clear();
            for (int b = r.first; b < r.second; b++)
                for (int lo = b * blk; lo < T; lo += L) lens.push_back(std::min(L, T - lo));
            std::sort(lens.begin(), lens.end(), std::greater<int>());
            std::priority_queue<double, std::vector<double>, std::greater<double>> q;
            for (int i = 0; i < slots; i++) q.push(0.0);
            double makespan = 0;
            for (int len : lens) {
                const double t = q.top() + len + fixed;
                q.pop();
                q.push(t);
                makespan = std::max(makespan, t);
            }
            cost += makespan;
        }
        if (cost < best_cost * (1.0 - 1e-9)) {
            best_cost = cost;
            best_L = L;
        }
        if (L >= 8192) break;
    }
    SymPlan p;
    p.blk = blk;
    p.chunk = best_L;
    p.nblk = nblk;
    std::vector<std::array<int32_t, 4>> all;   // (len, b, c, canon), block-major
    int32_t canon = 0;
    for (int b = 0; b < nblk; b++) {
        int c = 0;
        for (int lo = b * blk; lo < T; lo += best_L, c++)
            all.push_back({std::min(best_L, T - lo), b, c, canon++});
    }
    size_t e0 = 0;
    for (const auto &r : rounds) {
        const int b0 = r.first, b1 = r.second;
        size_t e1 = e0;
        while (e1 < all.size() && all[e1][1] < b1) e1++;
        std::vector<std::array<int32_t, 4>> rd(all.begin() + e0, all.begin() + e1);
        std::stable_sort(rd.begin(), rd.end(),
                         [](const std::array<int32_t, 4> &x, const std::array<int32_t, 4> &y) {
                             return x[0] > y[0];
                         });
        p.rounds.push_back(SymRound{b0, b1, (int)(p.items.size() / 3), (int)rd.size(),
                                    sym_sig_off(b0, T, blk)});
        for (const auto &e : rd) {
            p.items.push_back(e[1]);
            p.items.push_back(e[2]);
            p.items.push_back(e[3]);
        }
        p.sig_doubles = std::max(p.sig_doubles,
                                 (sym_sig_off(b1, T, blk) - sym_sig_off(b0, T, blk)) * SIG_VALS);
        e0 = e1;
    }
    p.tau_doubles = (int64_t)canon * blk * SIG_VALS;
    return cache.emplace(std::make_tuple(T, blk, slots, cap_mib), std::move(p)).first->second;
}

const SymPlan &sym_plan_for(const bem_mesh *m, const FarPlan &fp) {
    const void *k = fp.fr ? sym_kernel<true>(fp.code) : sym_kernel<false>(fp.code);
    return sym_plan((int)m->T, fp.blk, far_slots(k, fp.blk, far_smem<float>(fp.blk)));
}


}   // namespace

// right-hand sides per multi-vector pair-kernel launch
constexpr int FF_MULTI_MAX = 4;
constexpr int FF_MULTI_MAX_FP64 = 2;

// Upper bound over every block size and vectors-per-launch choice, so that
// it holds whatever the tuning table says.
int64_t farfield_scratch_bytes(const bem_mesh *m, int precision, double2 k0, double2 k1, int R) {
    const int64_t T = m->T;
    const bool f32 = precision == BEM_FP32;
    const int64_t rb = f32 ? 4 : 8;
    int64_t dyn = T * DYN_STRIDE * rb, part = 0;
    for (int blk : {64, 128, 256}) {
        const FarPlan p = far_plan(m, precision, k0, k1, blk);
        part = std::max(part, (int64_t)p.nsplit * T * (ROW_STRIDE + 6) * 8);
        if (f32) {
            const SymPlan &sp = sym_plan_for(m, p);
            part = std::max(part, (sp.tau_doubles + sp.sig_doubles + T * SIG_VALS) * 8 +
                                      (int64_t)sp.items.size() * 4);
        }
        if (R < 2 || (f32 && p.fr)) continue;
        for (int nr : {2, 4}) {
            if (nr > R || nr > (f32 ? FF_MULTI_MAX : FF_MULTI_MAX_FP64)) continue;
            const void *k = f32 ? (nr == 4 ? multi_kernel<float, 4>(p.code)
                                           : multi_kernel<float, 2>(p.code))
                                : multi_kernel<double, 2>(p.code);
            const int ns = farfield_splits((int)T, far_slots(k, blk, 0), blk);
            dyn = std::max(dyn, (int64_t)nr * T * DYN_STRIDE * rb);
            part = std::max(part, (int64_t)nr * ns * T * (ROW_STRIDE + 6) * 8);
        }
    }
    return dyn + part + T * ROW_STRIDE * 8;
}

void farfield_apply(bem_mesh *m, const NearOperator &nf, double2 k0, double2 k1,
                    double rho, const double2 *x, double2 *y, int precision,
                    hipStream_t s, int block) {
    const int T = (int)m->T;
    const FarPlan plan =
        far_plan(m, precision, k0, nf.k1_plan, valid_block(block > 0 ? block : tune_lookup(T, 1).block));
    const int blk = plan.blk;
    const int nsplit = plan.nsplit;
    const bool ck0 = k0.y != 0.0, ck1 = nf.k1_plan.y != 0.0, multi = m->nobj > 1, fr = plan.fr;
    const int split_len = (T + nsplit - 1) / nsplit;
    const bool sym = precision == BEM_FP32 && tuning().farfield_symmetric;
    const size_t need = (size_t)nsplit * T * (ROW_STRIDE + 6);
    if (!sym && m->partial.n < need) m->partial.alloc(need);
    if (m->trirows.n < (size_t)T * ROW_STRIDE) m->trirows.alloc((size_t)T * ROW_STRIDE);
    dim3 gg((T + 255) / 256);
    dim3 grid((T + blk - 1) / blk, nsplit);
    if (sym) {
        // each separated pair once, rows of both triangles
        if (m->dyn32.n < (size_t)T * DYN_STRIDE) m->dyn32.alloc((size_t)T * DYN_STRIDE);
        hipLaunchKernelGGL(source_gather_kernel<float>, gg, dim3(256), 0, s, m->tri_d.p,
                           m->tst.p, x, m->N, T, m->dyn32.p);
        BEM_LAUNCH_CHECK();
        const SymPlan &sp = sym_plan_for(m, plan);
        const size_t sneed = (size_t)(sp.tau_doubles + sp.sig_doubles + (int64_t)T * SIG_VALS);
        if (m->partial.n < sneed) m->partial.alloc(sneed);
        if (m->sym_items.n < sp.items.size() || m->sym_plan_id != &sp) {
            if (m->sym_items.n < sp.items.size()) m->sym_items.alloc(sp.items.size());
            BEM_HIP(hipMemcpyAsync(m->sym_items.p, sp.items.data(), sp.items.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, s));
            m->sym_plan_id = &sp;
        }
        double *ptau = m->partial.p, *psig = ptau + sp.tau_doubles, *sigacc = psig + sp.sig_doubles;
        const Coef<float> cf = make_coef<float>(k0, nf);
        const Int<float> *it = interior_table<float>(m, nf, k0);
        auto accum = [&](const SymRound &rd) {
            hipLaunchKernelGGL(sym_sig_accum_kernel, gg, dim3(256), 0, s, psig, rd.sig_base, rd.b0,
                               rd.b1, T, blk, sigacc);
            BEM_LAUNCH_CHECK();
        };
        {
            Timer tm("farfield_fp32", s);
            const size_t nr = sp.rounds.size();
            for (size_t r = 0; r < nr; r++) {
                const SymRound &rd = sp.rounds[r];
                const int32_t *items = m->sym_items.p + 3 * (int64_t)rd.item0;
                if (!fr)
                    launch_sym<false>(plan.code, rd.nitems, blk, s, m->geo32.p, m->dyn32.p,
                                      m->tobj_d.p, m->tri_d.p, T, items, sp.chunk, cf, it, ptau,
                                      psig, rd.sig_base);
                else
                    launch_sym<true>(plan.code, rd.nitems, blk, s, m->geo32.p, m->dyn32.p,
                                     m->tobj_d.p, m->tri_d.p, T, items, sp.chunk, cf, it, ptau,
                                     psig, rd.sig_base);
                BEM_LAUNCH_CHECK();
                if (r + 1 < nr) accum(rd);   // the slots are reused by the next round
            }
        }
        accum(sp.rounds.back());
        hipLaunchKernelGGL(reduce_sym_kernel, gg, dim3(256), 0, s, ptau, sigacc, m->tst.p, T, blk,
                           sp.chunk, m->trirows.p);
        BEM_LAUNCH_CHECK();
    } else if (precision == BEM_FP32) {
        if (m->dyn32.n < (size_t)T * DYN_STRIDE) m->dyn32.alloc((size_t)T * DYN_STRIDE);
        hipLaunchKernelGGL(source_gather_kernel<float>, gg, dim3(256), 0, s, m->tri_d.p,
                           m->tst.p, x, m->N, T, m->dyn32.p);
        BEM_LAUNCH_CHECK();
        Timer tm("farfield_fp32", s);
        if (!fr)
            dispatch_far<float, false>(grid, blk, s, m->geo32.p, m->dyn32.p, m->tobj_d.p, m->tri_d.p,
                                       T, split_len, make_coef<float>(k0, nf),
                                       interior_table<float>(m, nf, k0), m->partial.p, ck0, ck1,
                                       multi);
        else
            dispatch_far<float, true>(grid, blk, s, m->geo32.p, m->dyn32.p, m->tobj_d.p, m->tri_d.p,
                                      T, split_len, make_coef<float>(k0, nf),
                                      interior_table<float>(m, nf, k0), m->partial.p, ck0, ck1,
                                      multi);
        BEM_LAUNCH_CHECK();
    } else {
        if (m->dyn64.n < (size_t)T * DYN_STRIDE) m->dyn64.alloc((size_t)T * DYN_STRIDE);
        hipLaunchKernelGGL(source_gather_kernel<double>, gg, dim3(256), 0, s, m->tri_d.p,
                           m->tst.p, x, m->N, T, m->dyn64.p);
        BEM_LAUNCH_CHECK();
        Timer tm("farfield_fp64", s);
        dispatch_far<double, true>(grid, blk, s, m->geo64.p, m->dyn64.p, m->tobj_d.p, m->tri_d.p, T, split_len,
                             make_coef<double>(k0, nf), interior_table<double>(m, nf, k0), m->partial.p, ck0,
                             ck1, multi);
        BEM_LAUNCH_CHECK();
    }
    if (!sym) {
        hipLaunchKernelGGL(reduce_splits_kernel, gg, dim3(256), 0, s, m->partial.p, m->tst.p,
                           T, nsplit, m->trirows.p);
        BEM_LAUNCH_CHECK();
    }
    Timer tf("finalize", s);
    hipLaunchKernelGGL(finalize_kernel, dim3((m->N + 255) / 256), dim3(256), 0, s,
                       m->trirows.p, m->star_ptr.p, m->star_idx.p, m->nf_rowptr.p,
                       m->nf_col.p, (const double2 *)nf.vals.p, m->nf_nnz, x, m->N, y);
    BEM_LAUNCH_CHECK();
}

namespace {

// NR right-hand sides through the multi-vector kernel (FP32 without phase
// reduction, or FP64).
template <class R, int NR>
void farfield_multi_apply(bem_mesh *m, const NearOperator &nf, double2 k0, double2 k1,
                          double rho, int code, int blk, const double2 *x, double2 *y,
                          hipStream_t s) {
    constexpr bool F32 = std::is_same<R, float>::value;
    const int T = (int)m->T;
    const int64_t N = m->N, n2 = 2 * N;
    const int nsplit = farfield_splits(T, far_slots(multi_kernel<R, NR>(code), blk, 0), blk);
    const int split_len = (T + nsplit - 1) / nsplit;
    const int64_t rstride = (int64_t)nsplit * T * (ROW_STRIDE + 6);
    if (m->partial.n < (size_t)(NR * rstride)) m->partial.alloc((size_t)(NR * rstride));
    if (m->trirows.n < (size_t)T * ROW_STRIDE) m->trirows.alloc((size_t)T * ROW_STRIDE);
    R *dyn;
    if constexpr (F32) {
        if (m->dyn32.n < (size_t)NR * T * DYN_STRIDE) m->dyn32.alloc((size_t)NR * T * DYN_STRIDE);
        dyn = m->dyn32.p;
    } else {
        if (m->dyn64.n < (size_t)NR * T * DYN_STRIDE) m->dyn64.alloc((size_t)NR * T * DYN_STRIDE);
        dyn = m->dyn64.p;
    }
    const R *geo = F32 ? (const R *)m->geo32.p : (const R *)m->geo64.p;
    dim3 gg((T + 255) / 256);
    for (int r = 0; r < NR; r++) {
        hipLaunchKernelGGL(source_gather_kernel<R>, gg, dim3(256), 0, s, m->tri_d.p, m->tst.p,
                           x + r * n2, N, T, dyn + (int64_t)r * T * DYN_STRIDE);
        BEM_LAUNCH_CHECK();
    }
    {
        Timer tm(F32 ? "farfield_fp32_multi" : "farfield_fp64_multi", s);
        launch_multi<R, NR>(code, dim3((T + blk - 1) / blk, nsplit), blk, s, geo, dyn,
                            m->tobj_d.p, m->tri_d.p, T, split_len, make_coef<R>(k0, nf),
                            interior_table<R>(m, nf, k0), m->partial.p);
        BEM_LAUNCH_CHECK();
    }
    for (int r = 0; r < NR; r++) {
        hipLaunchKernelGGL(reduce_splits_kernel, gg, dim3(256), 0, s, m->partial.p + r * rstride,
                           m->tst.p, T, nsplit, m->trirows.p);
        BEM_LAUNCH_CHECK();
        hipLaunchKernelGGL(finalize_kernel, dim3((N + 255) / 256), dim3(256), 0, s, m->trirows.p,
                           m->star_ptr.p, m->star_idx.p, m->nf_rowptr.p, m->nf_col.p,
                           (const double2 *)nf.vals.p, m->nf_nnz, x + r * n2, N, y + r * n2);
        BEM_LAUNCH_CHECK();
    }
}

}   // namespace

void farfield_apply_batch(bem_mesh *m, const NearOperator &nf, double2 k0, double2 k1,
                          double rho, const double2 *x, double2 *y, int R, int precision,
                          hipStream_t s, const TuneEntry *forced) {
    const int64_t n2 = 2 * m->N;
    const TuneEntry te = forced ? *forced : tune_lookup(m->T, R);
    const int blk = valid_block(te.block);
    const FarPlan plan = far_plan(m, precision, k0, nf.k1_plan, blk);
    int r0 = 0;
    const int mm = te.multi;
    if (precision == BEM_FP32 && !plan.fr && mm >= 2) {
        if (mm >= 4)
            for (; R - r0 >= 4; r0 += 4)
                farfield_multi_apply<float, 4>(m, nf, k0, k1, rho, plan.code, blk, x + r0 * n2,
                                               y + r0 * n2, s);
        for (; R - r0 >= 2; r0 += 2)
            farfield_multi_apply<float, 2>(m, nf, k0, k1, rho, plan.code, blk, x + r0 * n2,
                                           y + r0 * n2, s);
    } else if (precision == BEM_FP64 && mm >= 2) {
        for (; R - r0 >= 2; r0 += 2)
            farfield_multi_apply<double, 2>(m, nf, k0, k1, rho, plan.code, blk, x + r0 * n2,
                                            y + r0 * n2, s);
    }
    for (; r0 < R; r0++)
        farfield_apply(m, nf, k0, k1, rho, x + r0 * n2, y + r0 * n2, precision, s, blk);
}

}   // namespace bem

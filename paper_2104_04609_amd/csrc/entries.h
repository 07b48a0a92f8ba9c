// Far-field entries of the permuted PMCHWT Galerkin operator (Sec. 2.7;
// operators of Sec. 2.2 with D in Maue form, P1 test and trial functions of
// Sec. 2.3) between one test triangle and the trial function of one vertex,
// shared by the dense assembly and the hierarchical (compressed) operator so
// that both hold the same numbers.
//
// tri_vertex_entries(tau, j): for the test functions a = 0..2 of tau, the
// sum over the trial triangles sigma of vertex j that share no vertex with
// tau of the 6x6-rule integrals of the four blocks against phi_j:
//   out[0 * 3 + a]  B11 = V_0 + rho V_1          (psi row, psi column)
//   out[1 * 3 + a]  B12 = -(K_0 + K_1)           (psi row, phi column)
//   out[2 * 3 + a]  B21 = K'_0 + K'_1            (phi row, psi column)
//   out[3 * 3 + a]  B22 = D_0 + D_1 / rho        (phi row, phi column)
// including the factor |tau| / (4 pi).  Pairs sharing a vertex belong to
// the FP64 near-field operator.
#pragma once

#include <type_traits>

#include "bem_internal.h"

namespace bem {
namespace entries {

constexpr double DUN_A1 = 0.44594849091596488631832925388305;
constexpr double DUN_W1 = 0.22338158967801146569500700843312;
constexpr double DUN_A2 = 0.091576213509770743459571463402202;
constexpr double DUN_W2 = 0.10995174365532186763832632490021;
__host__ __device__ constexpr double qw(int i) { return i < 3 ? DUN_W1 : DUN_W2; }
__host__ __device__ constexpr double qb(int i, int a) {
    return (a == i % 3) ? (1.0 - 2.0 * (i < 3 ? DUN_A1 : DUN_A2)) : (i < 3 ? DUN_A1 : DUN_A2);
}

// interior coefficients of one object (several objects: a per-object table)
template <class R> struct DIntT {
    R krev1, k1r, k1i, kdec1, rho, irho, n10r, n10i;
    R ns1;   // -s_1 (interior sign: +1 PMCHWT, -1 Mueller)
};
template <class R> struct DCoefT {
    R krev0, k0r, k0i, kdec0, n0r, n0i;
    DIntT<R> in;
};

__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Arithmetic per precision.  FP32: hardware sin/cos (in revolutions),
// 1/sqrt and exp2; stored as complex64.  FP64: sin/cos of 2 pi t from a table
// of e^{2 pi i n/256} and the Taylor series of the remainder (|2 pi f| <=
// pi/256, terms beyond x^6 below 4e-18), 1/sqrt from the hardware estimate and
// two Newton steps; complex128.
template <class R> struct DM;
template <> struct DM<float> {
    using C = float2;
    static __device__ __forceinline__ void fill_table(double2 *) {}
    static __device__ __forceinline__ void sincos(float t, float &s, float &c, const double2 *) {
        const float f = __builtin_amdgcn_fractf(t);   // hardware sin/cos take revolutions
        s = __builtin_amdgcn_sinf(f);
        c = __builtin_amdgcn_cosf(f);
    }
    static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float exp2(float x) { return __builtin_amdgcn_exp2f(x); }
    static __device__ __forceinline__ float2 mk(float a, float b) { return make_float2(a, b); }
};
template <> struct DM<double> {
    using C = double2;
    static __device__ __forceinline__ void fill_table(double2 *tab) {
        for (int n = threadIdx.x; n < 256; n += blockDim.x) {
            double sn, cs;
            ::sincos(n * (6.283185307179586476925286766559 / 256.0), &sn, &cs);
            tab[n] = make_double2(cs, sn);
        }
    }
    static __device__ __forceinline__ void sincos(double t, double &s, double &c,
                                                  const double2 *tab) {
        const double n = __builtin_rint(256.0 * t);
        const double x = __builtin_fma(-0.00390625, n, t) * 6.283185307179586476925286766559;
        const double x2 = x * x;
        const double sn = __builtin_fma(__builtin_fma(x2, 1.0 / 120.0, -1.0 / 6.0), x2, 1.0) * x;
        const double cs =
            __builtin_fma(__builtin_fma(__builtin_fma(x2, -1.0 / 720.0, 1.0 / 24.0), x2, -0.5), x2, 1.0);
        const double2 e = tab[((int64_t)n) & 255];
        c = __builtin_fma(e.x, cs, -e.y * sn);
        s = __builtin_fma(e.y, cs, e.x * sn);
    }
    static __device__ __forceinline__ double rsq(double x) {
        double y = __builtin_amdgcn_rsq(x);
        const double h = 0.5 * x;
        y = y * __builtin_fma(-h * y, y, 1.5);
        y = y * __builtin_fma(-h * y, y, 1.5);
        return y;
    }
    static __device__ __forceinline__ double exp2(double x) { return ::exp2(x); }
    static __device__ __forceinline__ double2 mk(double a, double b) { return make_double2(a, b); }
};

// Test triangle tau (geometry loaded by the caller: 6 points, normal, plane
// offset, curls), trial vertex j; out[blk * 3 + a] as above.  UNIFORM: every
// lane of the wave has the same j (interior coefficients of a trial triangle's
// object read once per wave).
template <class R, bool CK0, bool CK1, bool MULTI, bool UNIFORM>
__device__ __forceinline__ void tri_vertex_entries(
    const R *__restrict__ geo, const double *__restrict__ tst, const int32_t *__restrict__ tobj,
    const int32_t *__restrict__ tri, const int32_t *__restrict__ star_ptr,
    const int32_t *__restrict__ star_idx, int tt, int j, const R px[6], const R py[6],
    const R pz[6], R ntx, R nty, R ntz, R ct, const R cu[9], const DCoefT<R> &cf,
    const DIntT<R> *__restrict__ itab, const double2 *etab, R outr[12], R outi[12]) {
    using M = DM<R>;
    const int tv0 = tri[3 * tt], tv1 = tri[3 * tt + 1], tv2 = tri[3 * tt + 2];
    const int ot = MULTI ? tobj[tt] : 0;
    for (int c = 0; c < 12; c++) outr[c] = outi[c] = (R)0;
    const int e0 = star_ptr[j], e1 = star_ptr[j + 1];
    for (int e = e0; e < e1; e++) {
        const int sb = star_idx[e];
        const int s = sb / 3, b = sb - 3 * s;
        const int sv0 = tri[3 * s], sv1 = tri[3 * s + 1], sv2 = tri[3 * s + 2];
        const bool adj = sv0 == tv0 || sv0 == tv1 || sv0 == tv2 || sv1 == tv0 || sv1 == tv1 ||
                         sv1 == tv2 || sv2 == tv0 || sv2 == tv1 || sv2 == tv2;
        if (adj) continue;   // near field
        const R *h = geo + (int64_t)GEO_STRIDE * s;
        const R nsx = h[18], nsy = h[19], nsz = h[20], cs = h[21];
        const R as = (R)tst[TST_STRIDE * s];
        const R m1 = MULTI ? (tobj[s] == ot ? (R)1 : (R)0) : (R)1;
        // the interior part of sigma's object
        DIntT<R> c1;
        if constexpr (MULTI) {
            const int so = UNIFORM ? __builtin_amdgcn_readfirstlane(tobj[s]) : tobj[s];
            c1 = itab[so];
        } else {
            c1 = cf.in;
        }
        const R nn = ntx * nsx + nty * nsy + ntz * nsz;
        // factor of the G_N term taken out of the q sum: k_0^2 (n_x . n_y)
        const R gnr = cf.n0r * nn, gni = cf.n0i * nn;
        R tq[6], tx[6], dny[6];
        for (int q = 0; q < 6; q++) {
            tq[q] = (R)(qw(q) * qb(q, b)) * as;
            // (x - y).n_x = c_tau - y.n_tau, folded into the trial weight
            tx[q] = (ct - (h[3 * q] * ntx + h[3 * q + 1] * nty + h[3 * q + 2] * ntz)) * tq[q];
        }
        for (int p = 0; p < 6; p++) dny[p] = cs - (px[p] * nsx + py[p] * nsy + pz[p] * nsz);
        R gwr = (R)0, gwi = (R)0;
#pragma unroll
        for (int p = 0; p < 6; p++) {
            R vr = (R)0, vi = (R)0, fr = (R)0, fi = (R)0, kr = (R)0, ki = (R)0, nr = (R)0, ni = (R)0;
#pragma unroll
            for (int q = 0; q < 6; q++) {
                const R dx = h[3 * q] - px[p], dy = h[3 * q + 1] - py[p],
                        dz = h[3 * q + 2] - pz[p];
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R ri = M::rsq(r2);
                const R r = r2 * ri;
                // E_m = e^{i k_m r} (interior term masked across objects)
                R E0r, E0i, E1r, E1i;
                M::sincos(r * cf.krev0, E0i, E0r, etab);
                M::sincos(r * c1.krev1, E1i, E1r, etab);
                if (CK0) {
                    const R d0 = M::exp2(r * cf.kdec0);
                    E0r *= d0;
                    E0i *= d0;
                }
                if (CK1 || MULTI) {
                    R d1 = m1;
                    if (CK1) d1 *= M::exp2(r * c1.kdec1);
                    E1r *= d1;
                    E1i *= d1;
                }
                const R G0r = E0r * ri, G0i = E0i * ri, G1r = E1r * ri, G1i = E1i * ri;
                // F r^2 = i (k_0 E_0 + k_1 E_1) - G_0 - G_1
                R Fr = fmaR(c1.ns1, G1r, -G0r), Fi = fmaR(c1.ns1, G1i, -G0i);
                Fr = fmaR(-cf.k0r, E0i, Fr);
                Fi = fmaR(cf.k0r, E0r, Fi);
                Fr = fmaR(-c1.k1r, E1i, Fr);
                Fi = fmaR(c1.k1r, E1r, Fi);
                if (CK0) {
                    Fr = fmaR(-cf.k0i, E0r, Fr);
                    Fi = fmaR(-cf.k0i, E0i, Fi);
                }
                if (CK1) {
                    Fr = fmaR(-c1.k1i, E1r, Fr);
                    Fi = fmaR(-c1.k1i, E1i, Fi);
                }
                const R ri2 = ri * ri;
                Fr *= ri2;
                Fi *= ri2;
                const R t = tq[q];
                // V-row psi column: G_V t
                vr = fmaR(fmaR(c1.rho, G1r, G0r), t, vr);
                vi = fmaR(fmaR(c1.rho, G1i, G0i), t, vi);
                // V-row phi column: -(y - x).n_y F t (the factor after the q sum)
                fr = fmaR(Fr, t, fr);
                fi = fmaR(Fi, t, fi);
                // D-row psi column: F (x - y).n_x t
                kr = fmaR(Fr, tx[q], kr);
                ki = fmaR(Fi, tx[q], ki);
                // D-row phi column: -k_0^2 (n_x.n_y) (G_0 + k_1^2/(rho k_0^2) G_1) t
                R Nr = fmaR(c1.n10r, G1r, G0r), Ni = fmaR(c1.n10r, G1i, G0i);
                if (CK0 || CK1) {
                    Nr = fmaR(-c1.n10i, G1i, Nr);
                    Ni = fmaR(c1.n10i, G1r, Ni);
                }
                nr = fmaR(Nr, t, nr);
                ni = fmaR(Ni, t, ni);
                const R ww = (R)(qw(p) * qw(q));
                gwr = fmaR(ww, fmaR(c1.irho, G1r, G0r), gwr);
                gwi = fmaR(ww, fmaR(c1.irho, G1i, G0i), gwi);
            }
            // the four blocks at x_p, contracted at once with the test
            // functions (weights w_p phi_a(x_p)): no per-point state is kept
            const R v1r = -dny[p] * fr, v1i = -dny[p] * fi;
            const R v3r = -(gnr * nr - gni * ni), v3i = -(gnr * ni + gni * nr);
#pragma unroll
            for (int a = 0; a < 3; a++) {
                const R wp = (R)(qw(p) * qb(p, a));
                outr[a] = fmaR(wp, vr, outr[a]);
                outi[a] = fmaR(wp, vi, outi[a]);
                outr[3 + a] = fmaR(wp, v1r, outr[3 + a]);
                outi[3 + a] = fmaR(wp, v1i, outi[3 + a]);
                outr[6 + a] = fmaR(wp, kr, outr[6 + a]);
                outi[6 + a] = fmaR(wp, ki, outi[6 + a]);
                outr[9 + a] = fmaR(wp, v3r, outr[9 + a]);
                outi[9 + a] = fmaR(wp, v3i, outi[9 + a]);
            }
        }
        // curl-curl part of D
        R scb[3];
        for (int c = 0; c < 3; c++) scb[c] = (R)tst[TST_STRIDE * s + 1 + 3 * b + c];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const R cc = (cu[3 * a] * scb[0] + cu[3 * a + 1] * scb[1] + cu[3 * a + 2] * scb[2]) * as;
            outr[9 + a] += cc * gwr;
            outi[9 + a] += cc * gwi;
        }
    }
    const R sc = (R)(tst[TST_STRIDE * tt] * 0.079577471545947667884441881686257);
    for (int c = 0; c < 12; c++) {
        outr[c] *= sc;
        outi[c] *= sc;
    }
}

// Loads the test-side data of triangle tt for tri_vertex_entries.
template <class R>
__device__ __forceinline__ void load_test(const R *__restrict__ geo, const double *__restrict__ tst,
                                          int tt, R px[6], R py[6], R pz[6], R &ntx, R &nty,
                                          R &ntz, R &ct, R cu[9]) {
    const R *g = geo + (int64_t)GEO_STRIDE * tt;
    for (int i = 0; i < 6; i++) {
        px[i] = g[3 * i];
        py[i] = g[3 * i + 1];
        pz[i] = g[3 * i + 2];
    }
    ntx = g[18];
    nty = g[19];
    ntz = g[20];
    ct = g[21];
    for (int c = 0; c < 9; c++) cu[c] = (R)tst[TST_STRIDE * tt + 1 + c];
}

// s1 = -1 negates the interior terms (Mueller operator, Sec. 2.2): folded
// into rho, 1/rho, k_1^2/(rho k_0^2), k_1 (only in F) and ns1.
template <class R> inline DIntT<R> make_dint(double2 k0, double2 k1, double rho, int s1) {
    const double inv2pi = 0.15915494309189533576888376337251;
    const double log2e = 1.4426950408889634073599246810019;
    DIntT<R> c;
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

template <class R> inline DCoefT<R> make_dcoef(double2 k0, const NearOperator &nf) {
    const double inv2pi = 0.15915494309189533576888376337251;
    const double log2e = 1.4426950408889634073599246810019;
    DCoefT<R> c;
    c.krev0 = (R)(k0.x * inv2pi);
    c.k0r = (R)k0.x;
    c.k0i = (R)k0.y;
    c.kdec0 = (R)(-k0.y * log2e);
    c.n0r = (R)(k0.x * k0.x - k0.y * k0.y);
    c.n0i = (R)(2.0 * k0.x * k0.y);
    c.in = make_dint<R>(k0, nf.k1o[0], nf.rhoo[0], nf.s1);
    return c;
}

// Launch variant of a wavenumber pair: bit 2 complex k_0, bit 1 complex
// interior wavenumber, bit 0 several objects.
inline int variant_code(const bem_mesh *m, double2 k0, const NearOperator &nf) {
    return (k0.y != 0 ? 4 : 0) | (nf.k1_plan.y != 0 ? 2 : 0) | (m->nobj > 1 ? 1 : 0);
}

}   // namespace entries
}   // namespace bem

// Assembled form of the permuted PMCHWT Galerkin operator (Sec. 2.7;
// operators of Sec. 2.2, P1 Galerkin of Sec. 2.3) as a dense complex64
// matrix B [2N][2N] (row-major; rows [psi-row; phi-row] = [V-row; D-row],
// columns [psi; phi]), for right-hand-side batches and for GMRES iterations
// that reuse one operator many times.
//
// Entries are the same sums as the matrix-free matvec: the 6x6 rule (FP32)
// over every test/trial triangle pair sharing no vertex, plus the FP64
// near-field operator of the pairs that do.  Assembly is deterministic: per
// tile J of trial vertices,
//   dense_pairs_kernel:  Q[tau][j][a][blk] = sum_{sigma in star(j)} local
//                        block (tau, sigma)[a][b(sigma, j)]    (thread (tau, j))
//   dense_gather_kernel: B[i][j] = sum_{(tau, a) in star(i)} Q[tau][j][a]   (thread (i, j))
// Each separated triangle pair is evaluated three times (once per trial
// vertex), about three matrix-free matvecs of work per assembly.
#include <cmath>
#include <cstring>

#include "bem_internal.h"

namespace bem {

namespace {

constexpr double DUN_A1 = 0.44594849091596488631832925388305;
constexpr double DUN_W1 = 0.22338158967801146569500700843312;
constexpr double DUN_A2 = 0.091576213509770743459571463402202;
constexpr double DUN_W2 = 0.10995174365532186763832632490021;
__host__ __device__ constexpr double qw(int i) { return i < 3 ? DUN_W1 : DUN_W2; }
__host__ __device__ constexpr double qb(int i, int a) {
    return (a == i % 3) ? (1.0 - 2.0 * (i < 3 ? DUN_A1 : DUN_A2)) : (i < 3 ? DUN_A1 : DUN_A2);
}

typedef float fvec4 __attribute__((ext_vector_type(4)));

constexpr int JT = 512;   // trial vertices per assembly tile

// interior coefficients of one object (several objects: a per-object table)
struct DInt {
    float krev1, k1r, k1i, kdec1, rho, irho, n10r, n10i;
    float ns1;   // -s_1 (interior sign: +1 PMCHWT, -1 Mueller)
};
struct DCoef {
    float krev0, k0r, k0i, kdec0, n0r, n0i;
    DInt in;
};

__device__ __forceinline__ void sincos_rev(float t, float &s, float &c) {
    const float f = __builtin_amdgcn_fractf(t);   // hardware sin/cos take revolutions
    s = __builtin_amdgcn_sinf(f);
    c = __builtin_amdgcn_cosf(f);
}

template <bool CK0, bool CK1, bool MULTI>
__global__ __launch_bounds__(256) void dense_pairs_kernel(
    const float *__restrict__ geo, const double *__restrict__ tst,
    const int32_t *__restrict__ tobj, const int32_t *__restrict__ tri,
    const int32_t *__restrict__ star_ptr, const int32_t *__restrict__ star_idx, int T, int j0,
    int64_t N, DCoef cf, const DInt *__restrict__ itab, float2 *__restrict__ Q) {
    const int tau = blockIdx.x * 256 + threadIdx.x;
    const int jl = blockIdx.y;
    const int64_t j = j0 + jl;
    const bool active = tau < T && j < N;
    const int tt = tau < T ? tau : 0;
    const float *g = geo + (int64_t)GEO_STRIDE * tt;
    float px[6], py[6], pz[6];
    for (int i = 0; i < 6; i++) {
        px[i] = g[3 * i];
        py[i] = g[3 * i + 1];
        pz[i] = g[3 * i + 2];
    }
    const float ntx = g[18], nty = g[19], ntz = g[20], ct = g[21];
    const int tv0 = tri[3 * tt], tv1 = tri[3 * tt + 1], tv2 = tri[3 * tt + 2];
    const int ot = MULTI ? tobj[tt] : 0;
    float cu[9];
    for (int c = 0; c < 9; c++) cu[c] = (float)tst[TST_STRIDE * tt + 1 + c];
    float outr[12], outi[12];   // [blk * 3 + a]
    for (int c = 0; c < 12; c++) outr[c] = outi[c] = 0.f;
    const int e0 = j < N ? star_ptr[j] : 0, e1 = j < N ? star_ptr[j + 1] : 0;
    for (int e = e0; e < e1; e++) {
        const int sb = star_idx[e];
        const int s = sb / 3, b = sb - 3 * s;
        const int sv0 = tri[3 * s], sv1 = tri[3 * s + 1], sv2 = tri[3 * s + 2];
        const bool adj = sv0 == tv0 || sv0 == tv1 || sv0 == tv2 || sv1 == tv0 || sv1 == tv1 ||
                         sv1 == tv2 || sv2 == tv0 || sv2 == tv1 || sv2 == tv2;
        if (adj) continue;   // near field
        const float *h = geo + (int64_t)GEO_STRIDE * s;
        const float nsx = h[18], nsy = h[19], nsz = h[20], cs = h[21];
        const float as = (float)tst[TST_STRIDE * s];
        const float m1 = MULTI ? (tobj[s] == ot ? 1.f : 0.f) : 1.f;
        // sigma is the same for the whole block: its object's interior part
        const DInt c1 = MULTI ? itab[__builtin_amdgcn_readfirstlane(tobj[s])] : cf.in;
        const float nn = ntx * nsx + nty * nsy + ntz * nsz;
        // factor of the G_N term taken out of the q sum: k_0^2 (n_x . n_y)
        const float gnr = cf.n0r * nn, gni = cf.n0i * nn;
        float tq[6], tx[6], dny[6];
        for (int q = 0; q < 6; q++) {
            tq[q] = (float)(qw(q) * qb(q, b)) * as;
            // (x - y).n_x = c_tau - y.n_tau, folded into the trial weight
            tx[q] = (ct - (h[3 * q] * ntx + h[3 * q + 1] * nty + h[3 * q + 2] * ntz)) * tq[q];
        }
        for (int p = 0; p < 6; p++) dny[p] = cs - (px[p] * nsx + py[p] * nsy + pz[p] * nsz);
        float ar[4][6], ai[4][6];
        float gwr = 0.f, gwi = 0.f;
#pragma unroll
        for (int p = 0; p < 6; p++) {
            float vr = 0.f, vi = 0.f, fr = 0.f, fi = 0.f, kr = 0.f, ki = 0.f, nr = 0.f, ni = 0.f;
#pragma unroll
            for (int q = 0; q < 6; q++) {
                const float dx = h[3 * q] - px[p], dy = h[3 * q + 1] - py[p],
                            dz = h[3 * q + 2] - pz[p];
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float ri = __builtin_amdgcn_rsqf(r2);
                const float r = r2 * ri;
                // E_m = e^{i k_m r} (interior term masked across objects)
                float E0r, E0i, E1r, E1i;
                sincos_rev(r * cf.krev0, E0i, E0r);
                sincos_rev(r * c1.krev1, E1i, E1r);
                if (CK0) {
                    const float d0 = __builtin_amdgcn_exp2f(r * cf.kdec0);
                    E0r *= d0;
                    E0i *= d0;
                }
                if (CK1 || MULTI) {
                    float d1 = m1;
                    if (CK1) d1 *= __builtin_amdgcn_exp2f(r * c1.kdec1);
                    E1r *= d1;
                    E1i *= d1;
                }
                const float G0r = E0r * ri, G0i = E0i * ri, G1r = E1r * ri, G1i = E1i * ri;
                // F r^2 = i (k_0 E_0 + k_1 E_1) - G_0 - G_1
                float Fr = __builtin_fmaf(c1.ns1, G1r, -G0r), Fi = __builtin_fmaf(c1.ns1, G1i, -G0i);
                Fr = __builtin_fmaf(-cf.k0r, E0i, Fr);
                Fi = __builtin_fmaf(cf.k0r, E0r, Fi);
                Fr = __builtin_fmaf(-c1.k1r, E1i, Fr);
                Fi = __builtin_fmaf(c1.k1r, E1r, Fi);
                if (CK0) {
                    Fr = __builtin_fmaf(-cf.k0i, E0r, Fr);
                    Fi = __builtin_fmaf(-cf.k0i, E0i, Fi);
                }
                if (CK1) {
                    Fr = __builtin_fmaf(-c1.k1i, E1r, Fr);
                    Fi = __builtin_fmaf(-c1.k1i, E1i, Fi);
                }
                const float ri2 = ri * ri;
                Fr *= ri2;
                Fi *= ri2;
                const float t = tq[q];
                // V-row psi column: G_V t
                vr = __builtin_fmaf(__builtin_fmaf(c1.rho, G1r, G0r), t, vr);
                vi = __builtin_fmaf(__builtin_fmaf(c1.rho, G1i, G0i), t, vi);
                // V-row phi column: -(y - x).n_y F t (the factor after the q sum)
                fr = __builtin_fmaf(Fr, t, fr);
                fi = __builtin_fmaf(Fi, t, fi);
                // D-row psi column: F (x - y).n_x t
                kr = __builtin_fmaf(Fr, tx[q], kr);
                ki = __builtin_fmaf(Fi, tx[q], ki);
                // D-row phi column: -k_0^2 (n_x.n_y) (G_0 + k_1^2/(rho k_0^2) G_1) t
                float Nr = __builtin_fmaf(c1.n10r, G1r, G0r), Ni = __builtin_fmaf(c1.n10r, G1i, G0i);
                if (CK0 || CK1) {
                    Nr = __builtin_fmaf(-c1.n10i, G1i, Nr);
                    Ni = __builtin_fmaf(c1.n10i, G1r, Ni);
                }
                nr = __builtin_fmaf(Nr, t, nr);
                ni = __builtin_fmaf(Ni, t, ni);
                const float ww = (float)(qw(p) * qw(q));
                gwr = __builtin_fmaf(ww, __builtin_fmaf(c1.irho, G1r, G0r), gwr);
                gwi = __builtin_fmaf(ww, __builtin_fmaf(c1.irho, G1i, G0i), gwi);
            }
            ar[0][p] = vr;
            ai[0][p] = vi;
            ar[1][p] = -dny[p] * fr;
            ai[1][p] = -dny[p] * fi;
            ar[2][p] = kr;
            ai[2][p] = ki;
            ar[3][p] = -(gnr * nr - gni * ni);
            ai[3][p] = -(gnr * ni + gni * nr);
        }
        // contract with the test functions; curl-curl part of D
        float scb[3];
        for (int c = 0; c < 3; c++) scb[c] = (float)tst[TST_STRIDE * s + 1 + 3 * b + c];
#pragma unroll
        for (int a = 0; a < 3; a++) {
#pragma unroll
            for (int k = 0; k < 4; k++) {
                float sr = 0.f, si = 0.f;
#pragma unroll
                for (int p = 0; p < 6; p++) {
                    const float wp = (float)(qw(p) * qb(p, a));
                    sr += wp * ar[k][p];
                    si += wp * ai[k][p];
                }
                outr[3 * k + a] += sr;
                outi[3 * k + a] += si;
            }
            const float cc = (cu[3 * a] * scb[0] + cu[3 * a + 1] * scb[1] + cu[3 * a + 2] * scb[2]) * as;
            outr[9 + a] += cc * gwr;
            outi[9 + a] += cc * gwi;
        }
    }
    if (!active) return;
    const float sc = (float)(tst[TST_STRIDE * tt] * 0.079577471545947667884441881686257);
    float2 *o = Q + ((int64_t)tau * JT + jl) * 12;
    for (int c = 0; c < 12; c++) o[c] = make_float2(sc * outr[c], sc * outi[c]);
}

// B[i][j], B[i][N+j], B[N+i][j], B[N+i][N+j] from the star of test vertex i
__global__ __launch_bounds__(256) void dense_gather_kernel(const float2 *__restrict__ Q,
                                                           const int32_t *__restrict__ star_ptr,
                                                           const int32_t *__restrict__ star_idx,
                                                           int64_t N, int j0, int jt,
                                                           float2 *__restrict__ B) {
    const int jl = blockIdx.y * 256 + threadIdx.x;
    const int64_t i = blockIdx.x;
    if (jl >= jt) return;
    float2 acc[4] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
    for (int e = star_ptr[i]; e < star_ptr[i + 1]; e++) {
        const int ta = star_idx[e];
        const int t = ta / 3, a = ta - 3 * t;
        const float2 *q = Q + ((int64_t)t * JT + jl) * 12;
        for (int k = 0; k < 4; k++) {
            acc[k].x += q[3 * k + a].x;
            acc[k].y += q[3 * k + a].y;
        }
    }
    const int64_t n2 = 2 * N, j = j0 + jl;
    B[i * n2 + j] = acc[0];
    B[i * n2 + N + j] = acc[1];
    B[(N + i) * n2 + j] = acc[2];
    B[(N + i) * n2 + N + j] = acc[3];
}

// add the FP64 near-field operator (rounded to complex64)
__global__ __launch_bounds__(256) void dense_add_near_kernel(const int32_t *__restrict__ rowptr,
                                                             const int32_t *__restrict__ col,
                                                             const double2 *__restrict__ nf,
                                                             int64_t nnz, int64_t N,
                                                             float2 *__restrict__ B) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t n2 = 2 * N;
    for (int e = rowptr[i]; e < rowptr[i + 1]; e++) {
        const int64_t j = col[e];
        const int64_t pos[4] = {i * n2 + j, i * n2 + N + j, (N + i) * n2 + j,
                                (N + i) * n2 + N + j};
        for (int k = 0; k < 4; k++) {
            const double2 v = nf[k * nnz + e];
            float2 o = B[pos[k]];
            // sum in FP64, round once
            B[pos[k]] = make_float2((float)((double)o.x + v.x), (float)((double)o.y + v.y));
        }
    }
}

// y_r = B x_r for NR vectors (2..8); x: [NR][n2] complex64, y_r = y + r ystride.
// Two rows per wavefront (eight per
// workgroup); each chunk of the NR vectors (512 entries each) is staged in
// LDS once per workgroup and read by all eight rows, so x costs the L2 one
// pass per eight rows instead of one per row.  16-byte loads of B (2N even:
// rows and vectors 16-byte aligned), non-temporal; FP32 partial sums per
// chunk added in FP64, fixed-order wave reduction.
constexpr int GV_RW = 2;     // rows per wavefront
constexpr int GV_CH = 256;   // float4 (two complex entries) per chunk and vector

template <int NR>
__global__ __launch_bounds__(256) void dense_gemv_kernel(const float2 *__restrict__ B,
                                                         int64_t n2,
                                                         const float2 *__restrict__ x,
                                                         double2 *__restrict__ y,
                                                         int64_t ystride) {
    __shared__ fvec4 xs[NR * GV_CH];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * GV_RW;
    const int nrow = row0 >= n2 ? 0 : (n2 - row0 < GV_RW ? (int)(n2 - row0) : GV_RW);
    const fvec4 *b4[GV_RW];
    for (int q = 0; q < GV_RW; q++)
        b4[q] = reinterpret_cast<const fvec4 *>(B + (q < nrow ? row0 + q : 0) * n2);
    const fvec4 *x4 = reinterpret_cast<const fvec4 *>(x);
    const int64_t n4 = n2 / 2;
    double sr[GV_RW][NR], si[GV_RW][NR];
    for (int q = 0; q < GV_RW; q++)
        for (int r = 0; r < NR; r++) sr[q][r] = si[q][r] = 0.0;
    for (int64_t c0 = 0; c0 < n4; c0 += GV_CH) {
        const int cnt = n4 - c0 < GV_CH ? (int)(n4 - c0) : GV_CH;
        __syncthreads();   // the previous chunk's readers are done
        for (int idx = threadIdx.x; idx < NR * GV_CH; idx += 256) {
            const int r = idx / GV_CH, c = idx - r * GV_CH;
            xs[idx] = c < cnt ? x4[r * n4 + c0 + c] : fvec4{0.f, 0.f, 0.f, 0.f};
        }
        __syncthreads();
        if (nrow == 0) continue;   // (the barriers above stay uniform)
#pragma unroll
        for (int q = 0; q < GV_RW; q++) {
            fvec4 a[GV_CH / 64];
#pragma unroll
            for (int u = 0; u < GV_CH / 64; u++) {
                const int c = u * 64 + lane;
                a[u] = c < cnt ? __builtin_nontemporal_load(b4[q] + c0 + c)
                               : fvec4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int r = 0; r < NR; r++) {
                float pr = 0.f, pi = 0.f;
#pragma unroll
                for (int u = 0; u < GV_CH / 64; u++) {
                    const fvec4 v = xs[r * GV_CH + u * 64 + lane];
                    pr += a[u].x * v.x - a[u].y * v.y;
                    pi += a[u].x * v.y + a[u].y * v.x;
                    pr += a[u].z * v.z - a[u].w * v.w;
                    pi += a[u].z * v.w + a[u].w * v.z;
                }
                sr[q][r] += pr;
                si[q][r] += pi;
            }
        }
    }
    if (nrow == 0) return;
    for (int q = 0; q < GV_RW; q++)
        for (int r = 0; r < NR; r++)
            for (int o = 32; o > 0; o >>= 1) {
                sr[q][r] += __shfl_xor(sr[q][r], o, 64);
                si[q][r] += __shfl_xor(si[q][r], o, 64);
            }
    if (lane == 0)
        for (int q = 0; q < nrow; q++)
            for (int r = 0; r < NR; r++) y[r * ystride + row0 + q] = make_double2(sr[q][r], si[q][r]);
}

// y = B x for one vector: GEMV1_ROWS rows per wavefront (each chunk of x, read from
// cache, serves them all), 16-byte loads (two complex entries; 2N is even, so
// every row starts 16-byte aligned), eight loads of each row in flight per
// lane, B streamed with non-temporal loads.  FP32 partial sums over chunks
// of 1024 entries are added in FP64, then a fixed-order wave reduction.
constexpr int GEMV1_ROWS = 4;   // rows per wavefront

__global__ __launch_bounds__(256) void dense_gemv1_kernel(const float2 *__restrict__ B,
                                                          int64_t n2,
                                                          const float2 *__restrict__ x,
                                                          double2 *__restrict__ y) {
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * GEMV1_ROWS;
    const int lane = threadIdx.x & 63;
    if (row0 >= n2) return;
    const int nrow = n2 - row0 < GEMV1_ROWS ? (int)(n2 - row0) : GEMV1_ROWS;
    const fvec4 *b4[GEMV1_ROWS];
    for (int q = 0; q < GEMV1_ROWS; q++)
        b4[q] = reinterpret_cast<const fvec4 *>(B + (row0 + (q < nrow ? q : 0)) * n2);
    const fvec4 *x4 = reinterpret_cast<const fvec4 *>(x);
    const int64_t n4 = n2 / 2;
    double sr[GEMV1_ROWS], si[GEMV1_ROWS];
    for (int q = 0; q < GEMV1_ROWS; q++) sr[q] = si[q] = 0.0;
    int64_t c0 = 0;
    for (; c0 + 512 <= n4; c0 += 512) {
        fvec4 v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = x4[c0 + u * 64 + lane];
#pragma unroll
        for (int q = 0; q < GEMV1_ROWS; q++) {
            fvec4 a[8];
#pragma unroll
            for (int u = 0; u < 8; u++) a[u] = __builtin_nontemporal_load(b4[q] + c0 + u * 64 + lane);
            float pr = 0.f, pi = 0.f;
#pragma unroll
            for (int u = 0; u < 8; u++) {
                pr += a[u].x * v[u].x - a[u].y * v[u].y;
                pi += a[u].x * v[u].y + a[u].y * v[u].x;
                pr += a[u].z * v[u].z - a[u].w * v[u].w;
                pi += a[u].z * v[u].w + a[u].w * v[u].z;
            }
            sr[q] += pr;
            si[q] += pi;
        }
    }
    for (int q = 0; q < GEMV1_ROWS; q++) {
        float pr = 0.f, pi = 0.f;
        for (int64_t c = c0 + lane; c < n4; c += 64) {
            const fvec4 a = __builtin_nontemporal_load(b4[q] + c);
            const fvec4 v = x4[c];
            pr += a.x * v.x - a.y * v.y;
            pi += a.x * v.y + a.y * v.x;
            pr += a.z * v.z - a.w * v.w;
            pi += a.z * v.w + a.w * v.z;
        }
        sr[q] += pr;
        si[q] += pi;
    }
    for (int q = 0; q < GEMV1_ROWS; q++)
        for (int o = 32; o > 0; o >>= 1) {
            sr[q] += __shfl_xor(sr[q], o, 64);
            si[q] += __shfl_xor(si[q], o, 64);
        }
    if (lane == 0)
        for (int q = 0; q < nrow; q++) y[row0 + q] = make_double2(sr[q], si[q]);
}

// ------------------------------------------------ multi-RHS product on MFMA
// Y = B X for n_rhs right-hand sides as one real FP32 GEMM: B is read as a
// real [M][Kp] matrix (M = 2N rows, Kp = 4N: re/im interleaved), X as the
// real [Kp][Np] matrix with rows 2k = (Re X_k, Im X_k) and 2k+1 =
// (-Im X_k, Re X_k) per right-hand side (columns 2r, 2r+1), so that columns
// 2r and 2r+1 of the product are Re and Im of column r of B X.
constexpr int GM = 128, GN = 128, GK = 32;   // block tile and K step
constexpr int GKC = 4096;                    // split-K chunk (FP32 MFMA accumulation)

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Xp[2k][2r], Xp[2k][2r+1], Xp[2k+1][2r], Xp[2k+1][2r+1] from x[r][k] (RHS-major)
__global__ __launch_bounds__(256) void gemm_xprep_kernel(const double2 *__restrict__ x, int R,
                                                         int64_t K, int Np,
                                                         float *__restrict__ Xp) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= K * (Np / 2)) return;
    const int64_t k = id / (Np / 2);
    const int r = (int)(id - k * (Np / 2));
    const double2 v = r < R ? x[(int64_t)r * K + k] : make_double2(0.0, 0.0);
    float *row0 = Xp + (2 * k) * Np, *row1 = row0 + Np;
    row0[2 * r] = (float)v.x;
    row0[2 * r + 1] = (float)v.y;
    row1[2 * r] = (float)(-v.y);
    row1[2 * r + 1] = (float)v.x;
}

// partial products of K chunk blockIdx.z: Yp[z][M][Np]; 4 waves, 64 x 64 each.
// The next K step's tiles are loaded into registers (16-byte loads) while the
// current one is multiplied from LDS, then stored to the other LDS buffer:
// one barrier per K step.  Kp and Np are multiples of 4, chunk ends of 32.
__global__ __launch_bounds__(256) void gemm_mfma_kernel(const float *__restrict__ A,
                                                        const float *__restrict__ Xp,
                                                        float *__restrict__ Yp, int64_t M,
                                                        int64_t Kp, int Np) {
    __shared__ float As[2][GM][GK + 1];
    __shared__ float Bs[2][GK][GN];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * GM;
    const int n0 = blockIdx.y * GN;
    const int64_t kbeg = (int64_t)blockIdx.z * GKC;
    const int64_t kend = kbeg + GKC < Kp ? kbeg + GKC : Kp;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    floatx16 acc[2][2];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++)
            for (int v = 0; v < 16; v++) acc[i][j][v] = 0.f;
    // per thread: 4 float4 of the A tile (rows idx / 8, columns 4 (idx % 8)) and
    // 4 float4 of the B tile (rows idx / 32, columns 4 (idx % 32)), idx = i 256 + t
    float4 ra[4], rb[4];
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    auto gload = [&](int64_t k0) {
        for (int i = 0; i < 4; i++) {
            const int idx = i * 256 + t;
            const int64_t gr = m0 + idx / 8, gc = k0 + 4 * (idx % 8);
            ra[i] = (gr < M && gc < kend) ? *(const float4 *)(A + gr * Kp + gc) : zero4;
            const int64_t br = k0 + idx / 32;
            rb[i] = br < kend ? *(const float4 *)(Xp + br * Np + n0 + 4 * (idx % 32)) : zero4;
        }
    };
    auto lstore = [&](int buf) {
        for (int i = 0; i < 4; i++) {
            const int idx = i * 256 + t;
            float *a = &As[buf][idx / 8][4 * (idx % 8)];
            a[0] = ra[i].x;
            a[1] = ra[i].y;
            a[2] = ra[i].z;
            a[3] = ra[i].w;
            *(float4 *)&Bs[buf][idx / 32][4 * (idx % 32)] = rb[i];
        }
    };
    gload(kbeg);
    lstore(0);
    __syncthreads();
    int cur = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += GK) {
        const bool more = k0 + GK < kend;
        if (more) gload(k0 + GK);
#pragma unroll
        for (int kk = 0; kk < GK; kk += 2) {
            const int ka = kk + (lane >> 5);
            const float a0 = As[cur][wr + (lane & 31)][ka], a1 = As[cur][wr + 32 + (lane & 31)][ka];
            const float b0 = Bs[cur][ka][wc + (lane & 31)], b1 = Bs[cur][ka][wc + 32 + (lane & 31)];
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
        }
        if (more) lstore(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
    float *Y = Yp + (int64_t)blockIdx.z * M * Np;
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++)
            for (int v = 0; v < 16; v++) {
                // 32x32 accumulator layout: column lane % 32, row
                // 8 (v / 4) + 4 (lane / 32) + v % 4
                const int64_t row = m0 + wr + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int col = n0 + wc + 32 * j + (lane & 31);
                if (row < M) Y[row * Np + col] = acc[i][j][v];
            }
}

// y[r][m] = sum over K chunks (fixed order, FP64) of (Yp[.][m][2r], Yp[.][m][2r+1])
__global__ __launch_bounds__(256) void gemm_reduce_kernel(const float *__restrict__ Yp,
                                                          int nchunks, int64_t M, int Np, int R,
                                                          double2 *__restrict__ y) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= M * R) return;
    const int r = (int)(id / M);
    const int64_t m = id - (int64_t)r * M;
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < nchunks; c++) {
        const float *row = Yp + ((int64_t)c * M + m) * Np;
        sr += row[2 * r];
        si += row[2 * r + 1];
    }
    y[(int64_t)r * M + m] = make_double2(sr, si);
}

// ------------------------------------ 2-8 right-hand sides: skinny MFMA product
// The same real GEMM with 16 columns (8 complex right-hand sides) on
// v_mfma_f32_16x16x4f32.  HBM-bound: every wave streams blocks of 16 rows of
// B over its K chunk, 1 KB of each row per step, with load instructions that
// read 64 contiguous bytes of each of the 16 rows (the four lanes q of a row
// are adjacent): long per-row runs keep HBM streaming.  The operand is the
// transposed, re/im interleaved XT[16][Kp].  The 4 k-slots of an MFMA may
// hold any 4 values of k as long as A and XT agree: in a step of 256, lane
// (i, q) = (lane % 16, lane / 16) holds k = kb + 16c + 4q + e (c < 16, e < 4)
// and MFMA (c, e) takes component e of its c-th 16-byte load.
constexpr int SK_ROWS = 256;    // rows per workgroup (4 waves x 4 blocks of 16)
constexpr int SK_KC = 1024;     // split-K chunk (real K): FP32 accumulation length

typedef float floatx4 __attribute__((ext_vector_type(4)));

// XT[2r][2k], XT[2r][2k+1], XT[2r+1][2k], XT[2r+1][2k+1] from x[r][k], r < R <= 8
__global__ __launch_bounds__(256) void skinny_xprep_kernel(const double2 *__restrict__ x, int R,
                                                           int64_t K, float *__restrict__ XT) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= K * 8) return;
    const int r = (int)(id / K);
    const int64_t k = id - (int64_t)r * K;
    const double2 v = r < R ? x[(int64_t)r * K + k] : make_double2(0.0, 0.0);
    const int64_t Kp = 2 * K;
    float *re = XT + (2 * r) * Kp, *im = re + Kp;
    re[2 * k] = (float)v.x;
    re[2 * k + 1] = (float)(-v.y);
    im[2 * k] = (float)v.y;
    im[2 * k + 1] = (float)v.x;
}

// Yp[chunk][M][16] partial products; grid (ceil(M / 256), chunks).  The
// workgroup's XT chunk [16][SK_KC] is staged in LDS once; every wave streams
// 4 blocks of 16 rows, block by block, 1 KB of each row per step.
__global__ __launch_bounds__(256) void skinny_mfma_kernel(const float *__restrict__ A,
                                                          const float *__restrict__ XT,
                                                          float *__restrict__ Yp, int64_t M,
                                                          int64_t Kp) {
    // rows padded by 4 floats: the 16 rows' 16-byte reads fall in distinct banks
    constexpr int XS = SK_KC + 4;
    __shared__ float xs[16 * XS];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, q = lane >> 4;
    const int64_t kbeg = (int64_t)blockIdx.y * SK_KC;
    const int64_t kend = kbeg + SK_KC < Kp ? kbeg + SK_KC : Kp;
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int idx = threadIdx.x; idx < 16 * SK_KC / 4; idx += 256) {
        const int c = idx / (SK_KC / 4), k4 = 4 * (idx - c * (SK_KC / 4));
        *(float4 *)&xs[c * XS + k4] =
            kbeg + k4 < kend ? *(const float4 *)(XT + (int64_t)c * Kp + kbeg + k4) : zero4;
    }
    __syncthreads();
    floatx4 acc[4];
    for (int b = 0; b < 4; b++)
        for (int v = 0; v < 4; v++) acc[b][v] = 0.f;
    const int64_t rbase = (int64_t)blockIdx.x * SK_ROWS + wave * 64;
    // units u = (step, block): 16 rows x 256 k; the next unit's 16 loads are
    // issued before this unit's 64 MFMAs
    const int nsteps = (int)((kend - kbeg + 255) / 256);
    auto load = [&](int u, float4 (&a)[16]) {
        const int64_t kb = kbeg + 256 * (int64_t)(u >> 2);
        const int64_t row = rbase + 16 * (u & 3) + i;
        const bool rin = row < M;
        const float *arow = A + (rin ? row : 0) * Kp;
        for (int c = 0; c < 16; c++) {
            const int64_t kk = kb + 16 * c + 4 * q;   // multiple of 4, as are kend and Kp
            a[c] = (rin && kk < kend) ? *(const float4 *)(arow + kk) : zero4;
        }
    };
    float4 av[16], an[16], bv[16];
    load(0, av);
    for (int st = 0; st < nsteps; st++) {
        for (int c = 0; c < 16; c++)
            bv[c] = *(const float4 *)&xs[i * XS + 256 * st + 16 * c + 4 * q];
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const int u = 4 * st + b;
            const bool more = u + 1 < 4 * nsteps;
            if (more) load(u + 1, an);
            for (int c = 0; c < 16; c++) {
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[c].x, bv[c].x, acc[b], 0, 0, 0);
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[c].y, bv[c].y, acc[b], 0, 0, 0);
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[c].z, bv[c].z, acc[b], 0, 0, 0);
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[c].w, bv[c].w, acc[b], 0, 0, 0);
            }
            if (more)
                for (int c = 0; c < 16; c++) av[c] = an[c];
        }
    }
    // 16x16 accumulator layout: column lane % 16, row 4 (lane / 16) + v
    float *Y = Yp + (int64_t)blockIdx.y * M * 16;
    for (int b = 0; b < 4; b++) {
        const int64_t r0 = rbase + 16 * b + 4 * q;
        for (int v = 0; v < 4; v++)
            if (r0 + v < M) Y[(r0 + v) * 16 + i] = acc[b][v];
    }
}

__global__ __launch_bounds__(256) void to_c64_kernel(const double2 *__restrict__ x,
                                                     float2 *__restrict__ o, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = make_float2((float)x[i].x, (float)x[i].y);
}

// s1 = -1 negates the interior terms (Mueller operator, Sec. 2.2): folded
// into rho, 1/rho, k_1^2/(rho k_0^2), k_1 (only in F) and ns1.
DInt make_dint(double2 k0, double2 k1, double rho, int s1) {
    const double inv2pi = 0.15915494309189533576888376337251;
    const double log2e = 1.4426950408889634073599246810019;
    DInt c;
    c.krev1 = (float)(k1.x * inv2pi);
    c.k1r = (float)k1.x;
    c.k1i = (float)k1.y;
    c.kdec1 = (float)(-k1.y * log2e);
    c.rho = (float)rho;
    c.irho = (float)(1.0 / rho);
    // k_1^2 / (rho k_0^2); k_0 != 0 is checked at the entry points
    const double n0r = k0.x * k0.x - k0.y * k0.y, n0i = 2.0 * k0.x * k0.y;
    const double n1r = (k1.x * k1.x - k1.y * k1.y) / rho, n1i = 2.0 * k1.x * k1.y / rho;
    const double d = n0r * n0r + n0i * n0i;
    c.n10r = (float)((n1r * n0r + n1i * n0i) / d);
    c.n10i = (float)((n1i * n0r - n1r * n0i) / d);
    if (s1 < 0) {
        c.k1r = -c.k1r;
        c.k1i = -c.k1i;
        c.rho = -c.rho;
        c.irho = -c.irho;
        c.n10r = -c.n10r;
        c.n10i = -c.n10i;
    }
    c.ns1 = s1 < 0 ? 1.0f : -1.0f;
    return c;
}

DCoef make_dcoef(double2 k0, const NearOperator &nf) {
    const double inv2pi = 0.15915494309189533576888376337251;
    const double log2e = 1.4426950408889634073599246810019;
    DCoef c;
    c.krev0 = (float)(k0.x * inv2pi);
    c.k0r = (float)k0.x;
    c.k0i = (float)k0.y;
    c.kdec0 = (float)(-k0.y * log2e);
    c.n0r = (float)(k0.x * k0.x - k0.y * k0.y);
    c.n0i = (float)(2.0 * k0.x * k0.y);
    c.in = make_dint(k0, nf.k1o[0], nf.rhoo[0], nf.s1);
    return c;
}

template <bool A, bool B, bool C>
void launch_pairs(dim3 grid, hipStream_t s, bem_mesh *m, int j0, DCoef cf, const DInt *itab,
                  float2 *Q) {
    hipLaunchKernelGGL((dense_pairs_kernel<A, B, C>), grid, dim3(256), 0, s, m->geo32.p, m->tst.p,
                       m->tobj_d.p, m->tri_d.p, m->star_ptr.p, m->star_idx.p, (int)m->T, j0,
                       m->N, cf, itab, Q);
}

}   // namespace

int64_t dense_bytes(const bem_mesh *m) { return 4 * m->N * m->N * (int64_t)sizeof(float2); }
int64_t dense_assembly_scratch_bytes(const bem_mesh *m) {
    return m->T * (int64_t)JT * 12 * (int64_t)sizeof(float2) + 2 * m->N * (int64_t)sizeof(float2);
}

std::unique_ptr<DenseOperator> dense_assemble(bem_mesh *m, const NearOperator &nf, double2 k0,
                                              double2 k1, double rho, hipStream_t s) {
    auto op = std::make_unique<DenseOperator>();
    const int64_t N = m->N, n2 = 2 * N;
    op->n2 = n2;
    op->T = m->T;
    op->B.alloc((size_t)(n2 * n2));
    DevBuf<float2> Q((size_t)m->T * JT * 12);
    const DCoef cf = make_dcoef(k0, nf);
    DevBuf<float> itab;   // per-object interior parts (several objects)
    if (m->nobj > 1) {
        std::vector<float> h((size_t)m->nobj * (sizeof(DInt) / sizeof(float)));
        for (int o = 0; o < m->nobj; o++) {
            const DInt c = make_dint(k0, nf.k1o[o], nf.rhoo[o], nf.s1);
            std::memcpy(h.data() + (size_t)o * (sizeof(DInt) / sizeof(float)), &c, sizeof(c));
        }
        itab.upload(h);
    }
    const int code = (k0.y != 0 ? 4 : 0) | (nf.k1_plan.y != 0 ? 2 : 0) | (m->nobj > 1 ? 1 : 0);
    Timer tm("dense_assemble", s);
    for (int64_t j0 = 0; j0 < N; j0 += JT) {
        const int jt = (int)std::min<int64_t>(JT, N - j0);
        dim3 grid((unsigned)((m->T + 255) / 256), jt);
        switch (code) {
        case 0: launch_pairs<false, false, false>(grid, s, m, (int)j0, cf, (const DInt *)itab.p, Q.p); break;
        case 1: launch_pairs<false, false, true>(grid, s, m, (int)j0, cf, (const DInt *)itab.p, Q.p); break;
        case 2: launch_pairs<false, true, false>(grid, s, m, (int)j0, cf, (const DInt *)itab.p, Q.p); break;
        case 3: launch_pairs<false, true, true>(grid, s, m, (int)j0, cf, (const DInt *)itab.p, Q.p); break;
        case 4: launch_pairs<true, false, false>(grid, s, m, (int)j0, cf, (const DInt *)itab.p, Q.p); break;
        case 5: launch_pairs<true, false, true>(grid, s, m, (int)j0, cf, (const DInt *)itab.p, Q.p); break;
        case 6: launch_pairs<true, true, false>(grid, s, m, (int)j0, cf, (const DInt *)itab.p, Q.p); break;
        default: launch_pairs<true, true, true>(grid, s, m, (int)j0, cf, (const DInt *)itab.p, Q.p); break;
        }
        BEM_LAUNCH_CHECK();
        hipLaunchKernelGGL(dense_gather_kernel, dim3((unsigned)N, (jt + 255) / 256), dim3(256), 0,
                           s, Q.p, m->star_ptr.p, m->star_idx.p, N, (int)j0, jt, op->B.p);
        BEM_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(dense_add_near_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                       m->nf_rowptr.p, m->nf_col.p, (const double2 *)nf.vals.p, m->nf_nnz, N,
                       op->B.p);
    BEM_LAUNCH_CHECK();
    BEM_HIP(hipStreamSynchronize(s));   // Q is released on return
    return op;
}

template <int NR>
void launch_gemv(const DenseOperator &op, const float2 *xs, double2 *y, hipStream_t s) {
    hipLaunchKernelGGL(dense_gemv_kernel<NR>, dim3((unsigned)((op.n2 + 4 * GV_RW - 1) / (4 * GV_RW))),
                       dim3(256), 0, s, op.B.p, op.n2, xs, y, op.n2);
}

constexpr int GEMV_MAX_RHS = 8;   // right-hand sides per multi-vector GEMV launch

void dense_gemv(const DenseOperator &op, const double2 *x, double2 *y, int R, DevBuf<float2> &xs,
                hipStream_t s, bool skinny) {
    const int64_t n2 = op.n2;
    if (R == 1 || !skinny) {
        // multi-vector GEMV: one row per wavefront, B read once per 8 vectors
        const int64_t need = (int64_t)std::min(R, GEMV_MAX_RHS) * n2;
        if (xs.n < (size_t)need) xs.alloc((size_t)need);
        for (int r0 = 0; r0 < R; r0 += GEMV_MAX_RHS) {
            const int nr = std::min(GEMV_MAX_RHS, R - r0);
            const int64_t cnt = nr * n2;
            hipLaunchKernelGGL(to_c64_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                               s, x + r0 * n2, xs.p, cnt);
            BEM_LAUNCH_CHECK();
            Timer tm("dense_gemv", s);
            double2 *yr = y + r0 * n2;
            switch (nr) {
            case 1:
                hipLaunchKernelGGL(dense_gemv1_kernel,
                                   dim3((unsigned)((n2 + 4 * GEMV1_ROWS - 1) / (4 * GEMV1_ROWS))),
                                   dim3(256), 0, s, op.B.p, n2, xs.p, yr);
                break;
            case 2: launch_gemv<2>(op, xs.p, yr, s); break;
            case 3: launch_gemv<3>(op, xs.p, yr, s); break;
            case 4: launch_gemv<4>(op, xs.p, yr, s); break;
            case 5: launch_gemv<5>(op, xs.p, yr, s); break;
            case 6: launch_gemv<6>(op, xs.p, yr, s); break;
            case 7: launch_gemv<7>(op, xs.p, yr, s); break;
            default: launch_gemv<8>(op, xs.p, yr, s); break;
            }
            BEM_LAUNCH_CHECK();
        }
        return;
    }
    const int64_t M = n2, Kp = 2 * n2;
    const int nchunks = (int)((Kp + SK_KC - 1) / SK_KC);
    DevBuf<float> XT((size_t)(16 * Kp));
    DevBuf<float> Yp((size_t)nchunks * M * 16);
    for (int r0 = 0; r0 < R; r0 += 8) {
        const int nr = std::min(8, R - r0);
        hipLaunchKernelGGL(skinny_xprep_kernel, dim3((unsigned)((8 * n2 + 255) / 256)), dim3(256),
                           0, s, x + r0 * n2, nr, n2, XT.p);
        BEM_LAUNCH_CHECK();
        {
            Timer tm("dense_skinny_mfma", s);
            hipLaunchKernelGGL(skinny_mfma_kernel,
                               dim3((unsigned)((M + SK_ROWS - 1) / SK_ROWS), nchunks), dim3(256),
                               0, s, (const float *)op.B.p, XT.p, Yp.p, M, Kp);
            BEM_LAUNCH_CHECK();
        }
        const int64_t red = M * nr;
        hipLaunchKernelGGL(gemm_reduce_kernel, dim3((unsigned)((red + 255) / 256)), dim3(256), 0, s,
                           Yp.p, nchunks, M, 16, nr, y + r0 * n2);
        BEM_LAUNCH_CHECK();
    }
    BEM_HIP(hipStreamSynchronize(s));   // XT, Yp are released on return
}

int64_t dense_gemm_scratch_bytes(const bem_mesh *m, int R) {
    const int64_t M = 2 * m->N, Kp = 2 * M;
    const int64_t Np = 2 * (((int64_t)R + 63) / 64) * 64, nchunks = (Kp + GKC - 1) / GKC;
    return (Kp * Np + nchunks * M * Np) * (int64_t)sizeof(float);
}

void dense_apply(const DenseOperator &op, const double2 *x, double2 *y, int R,
                 DevBuf<float2> &xs, hipStream_t s, const TuneEntry *forced) {
    const TuneEntry te = forced ? *forced : tune_lookup(op.T, R);
    if (R >= te.gemm_min) dense_gemm(op, x, y, R, s);
    else dense_gemv(op, x, y, R, xs, s, R >= te.skinny_min);
}

void dense_gemm(const DenseOperator &op, const double2 *x, double2 *y, int R, hipStream_t s) {
    const int64_t M = op.n2, K = op.n2, Kp = 2 * K;
    const int Rp = ((R + 63) / 64) * 64, Np = 2 * Rp;
    const int nchunks = (int)((Kp + GKC - 1) / GKC);
    DevBuf<float> Xp((size_t)(Kp * Np));
    DevBuf<float> Yp((size_t)nchunks * M * Np);
    const int64_t prep = K * Rp;
    hipLaunchKernelGGL(gemm_xprep_kernel, dim3((unsigned)((prep + 255) / 256)), dim3(256), 0, s, x,
                       R, K, Np, Xp.p);
    BEM_LAUNCH_CHECK();
    {
        Timer tm("dense_gemm_mfma", s);
        hipLaunchKernelGGL(gemm_mfma_kernel,
                           dim3((unsigned)((M + GM - 1) / GM), Np / GN, nchunks), dim3(256), 0, s,
                           (const float *)op.B.p, Xp.p, Yp.p, M, Kp, Np);
        BEM_LAUNCH_CHECK();
    }
    const int64_t red = M * R;
    hipLaunchKernelGGL(gemm_reduce_kernel, dim3((unsigned)((red + 255) / 256)), dim3(256), 0, s,
                       Yp.p, nchunks, M, Np, R, y);
    BEM_LAUNCH_CHECK();
    BEM_HIP(hipStreamSynchronize(s));   // Xp, Yp are released on return
}

const DenseOperator &dense_get(bem_mesh *m, double2 k0, double2 k1, double rho, hipStream_t s,
                               int s1, const ObjMaterials *om) {
    const NearKey key = near_key(m, k0, k1, rho, s1, om);
    auto it = m->dense_cache.find(key);
    if (it != m->dense_cache.end()) return *it->second;
    const NearOperator &nf = nearfield_get(m, k0, k1, rho, s, s1, om);
    // one resident dense operator per mesh unless memory allows more
    size_t free_b = 0, total_b = 0;
    BEM_HIP(hipMemGetInfo(&free_b, &total_b));
    while (!m->dense_cache.empty() && (int64_t)free_b < dense_bytes(m) + (int64_t)(1ll << 30)) {
        m->dense_cache.erase(m->dense_cache.begin());
        BEM_HIP(hipMemGetInfo(&free_b, &total_b));
    }
    if ((int64_t)free_b < dense_bytes(m) + (int64_t)(1ll << 30))
        fail(BEM_E_NOMEM, "dense operator of " + std::to_string(dense_bytes(m)) +
                              " bytes does not fit in device memory");
    auto op = dense_assemble(m, nf, k0, k1, rho, s);
    auto &ref = *op;
    m->dense_cache.emplace(key, std::move(op));
    return ref;
}

}   // namespace bem

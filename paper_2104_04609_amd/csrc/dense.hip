// Assembled form of the permuted PMCHWT Galerkin operator (Sec. 2.7;
// operators of Sec. 2.2, P1 Galerkin of Sec. 2.3) as a dense complex64
// matrix B [2N][2N] (row-major; rows [psi-row; phi-row] = [V-row; D-row],
// columns [psi; phi]), for right-hand-side batches and for GMRES iterations
// that reuse one operator many times.
//
// Entries are the same sums as the matrix-free matvec: the 6x6 rule (FP32)
// over every test/trial triangle pair sharing no vertex, plus the FP64
// near-field operator of the pairs that do.
//
// The far part is symmetric under exchange of test and trial functions (the
// same rule on both sides, a kernel symmetric in x and y): V and D are
// symmetric and K' = K^T, so B[j][i] = B[i][j], B[N+j][N+i] = B[N+i][N+j] and
// B[N+j][i] = -B[i][N+j].  Only the entries with rank(i) <= rank(j) are
// evaluated, rank being the vertex's place in a Morton order of the vertex
// coordinates (vertices of one triangle get close ranks, so that about half
// of the work remains); dense_mirror_kernel fills in the others.  Per tile J
// of trial vertices (consecutive ranks),
//   dense_pairs_kernel:  Q[tau][j][a][blk] = sum_{sigma in star(j)} local
//                        block (tau, sigma)[a][b(sigma, j)]    (thread (tau, j),
//                        only where min rank(tau) <= rank(j))
//   dense_gather_kernel: B[i][j] = sum_{(tau, a) in star(i)} Q[tau][j][a]   (thread (i, j),
//                        only where rank(i) <= rank(j))
// Each separated triangle pair is evaluated about 1.5 times (three times for
// every trial vertex without the symmetry); assembly is deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "bem_internal.h"
#include "entries.h"

namespace bem {

namespace {

using namespace entries;

typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef double dvec2 __attribute__((ext_vector_type(2)));

constexpr int JT = 512;   // trial vertices per assembly tile

// At least two waves per SIMD: the FP64 instance otherwise takes 256 VGPRs
// plus AGPRs (one wave per SIMD); with the limit it keeps about 20 values in
// scratch and assembles 15 % faster.  The FP32 instances (143 VGPRs) run at 3.
template <class R, bool CK0, bool CK1, bool MULTI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void dense_pairs_kernel(
    const R *__restrict__ geo, const double *__restrict__ tst,
    const int32_t *__restrict__ tobj, const int32_t *__restrict__ tri,
    const int32_t *__restrict__ star_ptr, const int32_t *__restrict__ star_idx,
    const int32_t *__restrict__ order, int n_tau, const int32_t *__restrict__ rank,
    const int32_t *__restrict__ byrank, int T, int r0, int64_t N, DCoefT<R> cf,
    const DIntT<R> *__restrict__ itab, typename DM<R>::C *__restrict__ Q) {
    using M = DM<R>;
    __shared__ double2 etab[std::is_same<R, double>::value ? 256 : 1];   // FP64 sin/cos table
    M::fill_table(etab);
    __syncthreads();
    // test triangles in ascending order of their smallest vertex rank: the
    // first n_tau of them have a vertex ranked inside or before this tile
    const int k = blockIdx.x * 256 + threadIdx.x;
    const int tau = k < n_tau ? order[k] : T;
    const int jl = blockIdx.y;
    const int rj = r0 + jl;
    const int j = rj < N ? byrank[rj] : 0;
    const int tt = tau < T ? tau : 0;
    const int tv0 = tri[3 * tt], tv1 = tri[3 * tt + 1], tv2 = tri[3 * tt + 2];
    // Q[tau][j] is read only for rows i of tau with rank(i) <= rank(j)
    const bool active = tau < T && rj < N &&
                        min(rank[tv0], min(rank[tv1], rank[tv2])) <= rj;
    if (!active) return;
    R px[6], py[6], pz[6], ntx, nty, ntz, ct, cu[9];
    load_test(geo, tst, tt, px, py, pz, ntx, nty, ntz, ct, cu);
    R outr[12], outi[12];   // [blk * 3 + a]
    tri_vertex_entries<R, CK0, CK1, MULTI, true>(geo, tst, tobj, tri, star_ptr, star_idx, tt, j,
                                                 px, py, pz, ntx, nty, ntz, ct, cu, cf, itab,
                                                 etab, outr, outi);
    typename M::C *o = Q + ((int64_t)tau * JT + jl) * 12;
    for (int c = 0; c < 12; c++) o[c] = M::mk(outr[c], outi[c]);
}

// B[i][j], B[i][N+j], B[N+i][j], B[N+i][N+j] from the star of test vertex i,
// for the trial vertices j of the tile with rank(j) >= rank(i)
template <class C>
__global__ __launch_bounds__(256) void dense_gather_kernel(const C *__restrict__ Q,
                                                           const int32_t *__restrict__ star_ptr,
                                                           const int32_t *__restrict__ star_idx,
                                                           const int32_t *__restrict__ rank,
                                                           const int32_t *__restrict__ byrank,
                                                           int64_t N, int r0, int jt,
                                                           C *__restrict__ B) {
    const int jl = blockIdx.y * 256 + threadIdx.x;
    const int64_t i = blockIdx.x;
    if (jl >= jt || rank[i] > r0 + jl) return;
    C acc[4];
    for (int k = 0; k < 4; k++) acc[k].x = acc[k].y = 0;
    for (int e = star_ptr[i]; e < star_ptr[i + 1]; e++) {
        const int ta = star_idx[e];
        const int t = ta / 3, a = ta - 3 * t;
        const C *q = Q + ((int64_t)t * JT + jl) * 12;
        for (int k = 0; k < 4; k++) {
            acc[k].x += q[3 * k + a].x;
            acc[k].y += q[3 * k + a].y;
        }
    }
    const int64_t n2 = 2 * N, j = byrank[r0 + jl];
    B[i * n2 + j] = acc[0];
    B[i * n2 + N + j] = acc[1];
    B[(N + i) * n2 + j] = acc[2];
    B[(N + i) * n2 + N + j] = acc[3];
}

// Entries with rank(i) > rank(j) from their mirror images (blockIdx.z picks
// the block): B[i][j] = B[j][i], B[N+i][N+j] = B[N+j][N+i],
// B[N+i][j] = -B[j][N+i], B[i][N+j] = -B[N+j][i].  32 x 32 tiles transposed
// through LDS; the entries read are never written here (their row ranks lower).
template <class C>
__global__ __launch_bounds__(256) void dense_mirror_kernel(const int32_t *__restrict__ rank,
                                                           int64_t N, C *__restrict__ B) {
    __shared__ C tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t I0 = (int64_t)blockIdx.x * 32, J0 = (int64_t)blockIdx.y * 32;
    const int64_t n2 = 2 * N;
    const int z = blockIdx.z;
    const int64_t ro = (z == 0 || z == 2) ? 0 : N;   // row offset of the entries read
    const int64_t co = (z == 0 || z == 3) ? 0 : N;   // column offset of the entries read
    const float sg = z < 2 ? 1.0f : -1.0f;
    // read B[ro + j][co + i] for j in the J tile, i in the I tile
    const int64_t ic = I0 + tx;
    const int ri = ic < N ? rank[ic] : 0;
    for (int rr = 0; rr < 32; rr += 8) {
        const int64_t jr = J0 + ty + rr;
        C v;
        v.x = v.y = 0;
        if (jr < N && ic < N && rank[jr] < ri) v = B[(ro + jr) * n2 + co + ic];
        tile[ty + rr][tx] = v;
    }
    __syncthreads();
    // write B[co + i][ro + j] for i in the I tile, j in the J tile
    const int64_t jc = J0 + tx;
    const int rjc = jc < N ? rank[jc] : 0;
    for (int rr = 0; rr < 32; rr += 8) {
        const int64_t ir = I0 + ty + rr;
        if (ir < N && jc < N && rank[ir] > rjc) {
            C v = tile[tx][ty + rr];
            v.x *= sg;
            v.y *= sg;
            B[(co + ir) * n2 + ro + jc] = v;
        }
    }
}

// add the FP64 near-field operator (complex64: summed in FP64, rounded once)
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
            B[pos[k]] = make_float2((float)((double)o.x + v.x), (float)((double)o.y + v.y));
        }
    }
}

__global__ __launch_bounds__(256) void dense_add_near64_kernel(const int32_t *__restrict__ rowptr,
                                                               const int32_t *__restrict__ col,
                                                               const double2 *__restrict__ nf,
                                                               int64_t nnz, int64_t N,
                                                               double2 *__restrict__ B) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t n2 = 2 * N;
    for (int e = rowptr[i]; e < rowptr[i + 1]; e++) {
        const int64_t j = col[e];
        const int64_t pos[4] = {i * n2 + j, i * n2 + N + j, (N + i) * n2 + j,
                                (N + i) * n2 + N + j};
        for (int k = 0; k < 4; k++) {
            const double2 v = nf[k * nnz + e];
            B[pos[k]].x += v.x;
            B[pos[k]].y += v.y;
        }
    }
}

// y = B x with the complex128 operator, one vector: two rows per wavefront,
// 16-byte loads (one complex entry), eight per row in flight per lane, B
// streamed with non-temporal loads; FP64 sums, fixed-order wave reduction.
constexpr int G64_RW = 2;
__global__ __launch_bounds__(256) void dense_gemv64_kernel(const double2 *__restrict__ B,
                                                           int64_t n2,
                                                           const double2 *__restrict__ x,
                                                           double2 *__restrict__ y) {
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * G64_RW;
    const int lane = threadIdx.x & 63;
    if (row0 >= n2) return;
    const int nrow = n2 - row0 < G64_RW ? (int)(n2 - row0) : G64_RW;
    const dvec2 *b[G64_RW];
    for (int q = 0; q < G64_RW; q++)
        b[q] = reinterpret_cast<const dvec2 *>(B + (row0 + (q < nrow ? q : 0)) * n2);
    double sr[G64_RW], si[G64_RW];
    for (int q = 0; q < G64_RW; q++) sr[q] = si[q] = 0.0;
    int64_t c0 = 0;
    for (; c0 + 512 <= n2; c0 += 512) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = x[c0 + u * 64 + lane];
#pragma unroll
        for (int q = 0; q < G64_RW; q++) {
            dvec2 a[8];
#pragma unroll
            for (int u = 0; u < 8; u++) a[u] = __builtin_nontemporal_load(b[q] + c0 + u * 64 + lane);
#pragma unroll
            for (int u = 0; u < 8; u++) {
                sr[q] = __builtin_fma(a[u].x, v[u].x, __builtin_fma(-a[u].y, v[u].y, sr[q]));
                si[q] = __builtin_fma(a[u].x, v[u].y, __builtin_fma(a[u].y, v[u].x, si[q]));
            }
        }
    }
    for (int q = 0; q < G64_RW; q++)
        for (int64_t c = c0 + lane; c < n2; c += 64) {
            const dvec2 a = __builtin_nontemporal_load(b[q] + c);
            const double2 v = x[c];
            sr[q] = __builtin_fma(a.x, v.x, __builtin_fma(-a.y, v.y, sr[q]));
            si[q] = __builtin_fma(a.x, v.y, __builtin_fma(a.y, v.x, si[q]));
        }
    for (int q = 0; q < G64_RW; q++)
        for (int o = 32; o > 0; o >>= 1) {
            sr[q] += __shfl_xor(sr[q], o, 64);
            si[q] += __shfl_xor(si[q], o, 64);
        }
    if (lane == 0)
        for (int q = 0; q < nrow; q++) y[row0 + q] = make_double2(sr[q], si[q]);
}

// y_r = B x_r for NR vectors (2..8); x: [NR][n2] complex64, y_r = y + r ystride.
// Two rows per wavefront, GV_WAVES wavefronts per workgroup; each chunk of the
// NR vectors (512 entries each) is staged in LDS once per workgroup and read by
// all its rows (each LDS value once per wavefront, for both of its rows), so x
// costs the L2 one pass per 2 GV_WAVES rows.  16-byte loads of B (2N even:
// rows and vectors 16-byte aligned), non-temporal; FP32 partial sums per chunk
// added in FP64, fixed-order wave reduction.
constexpr int GV_RW = 2;      // rows per wavefront
constexpr int GV_CH = 256;    // float4 (two complex entries) per chunk and vector
constexpr int GV_WAVES = 8;   // wavefronts per workgroup

template <int NR>
__global__ __launch_bounds__(64 * GV_WAVES) void dense_gemv_kernel(const float2 *__restrict__ B,
                                                                   int64_t n2,
                                                                   const float2 *__restrict__ x,
                                                                   double2 *__restrict__ y,
                                                                   int64_t ystride) {
    constexpr int NT = 64 * GV_WAVES, NU = GV_CH / 64;
    __shared__ fvec4 xs[NR * GV_CH];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t row0 = ((int64_t)blockIdx.x * GV_WAVES + wave) * GV_RW;
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
        for (int idx = threadIdx.x; idx < NR * GV_CH; idx += NT) {
            const int r = idx / GV_CH, c = idx - r * GV_CH;
            xs[idx] = c < cnt ? x4[r * n4 + c0 + c] : fvec4{0.f, 0.f, 0.f, 0.f};
        }
        __syncthreads();
        if (nrow == 0) continue;   // (the barriers above stay uniform)
        fvec4 a[GV_RW][NU];
#pragma unroll
        for (int q = 0; q < GV_RW; q++)
#pragma unroll
            for (int u = 0; u < NU; u++) {
                const int c = u * 64 + lane;
                a[q][u] = c < cnt ? __builtin_nontemporal_load(b4[q] + c0 + c)
                                  : fvec4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
        for (int r = 0; r < NR; r++) {
            float pr[GV_RW], pi[GV_RW];
#pragma unroll
            for (int q = 0; q < GV_RW; q++) pr[q] = pi[q] = 0.f;
#pragma unroll
            for (int u = 0; u < NU; u++) {
                const fvec4 v = xs[r * GV_CH + u * 64 + lane];
#pragma unroll
                for (int q = 0; q < GV_RW; q++) {
                    pr[q] += a[q][u].x * v.x - a[q][u].y * v.y;
                    pi[q] += a[q][u].x * v.y + a[q][u].y * v.x;
                    pr[q] += a[q][u].z * v.z - a[q][u].w * v.w;
                    pi[q] += a[q][u].z * v.w + a[q][u].w * v.z;
                }
            }
#pragma unroll
            for (int q = 0; q < GV_RW; q++) {
                sr[q][r] += pr[q];
                si[q][r] += pi[q];
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
constexpr int GKC = 4096;                    // largest split-K chunk (FP32 MFMA accumulation)
constexpr int GKC_MIN = 1024;                // smallest split-K chunk

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
                                                        int64_t Kp, int Np, int kchunk) {
    __shared__ float As[2][GM][GK + 1];
    __shared__ float Bs[2][GK][GN];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * GM;
    const int n0 = blockIdx.y * GN;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = kbeg + kchunk < Kp ? kbeg + kchunk : Kp;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int v = 0; v < 16; v++) acc[i][j][v] = 0.f;
    // per thread: 4 float4 of the A tile (rows idx / 8, columns 4 (idx % 8)) and
    // 4 float4 of the B tile (rows idx / 32, columns 4 (idx % 32)), idx = i 256 + t,
    // held in named registers (no local array)
    float4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
#define BEM_GEMM_LOAD_ONE(i, RA, RB)                                                            \
    {                                                                                          \
        const int idx = (i) * 256 + t;                                                         \
        const int64_t gr = m0 + idx / 8, gc = k0 + 4 * (idx % 8);                              \
        RA = (gr < M && gc < kend) ? *(const float4 *)(A + gr * Kp + gc) : zero4;              \
        const int64_t br = k0 + idx / 32;                                                      \
        RB = br < kend ? *(const float4 *)(Xp + br * Np + n0 + 4 * (idx % 32)) : zero4;        \
    }
#define BEM_GEMM_STORE_ONE(i, RA, RB)                                                           \
    {                                                                                          \
        const int idx = (i) * 256 + t;                                                         \
        float *a = &As[buf][idx / 8][4 * (idx % 8)];                                           \
        a[0] = RA.x;                                                                           \
        a[1] = RA.y;                                                                           \
        a[2] = RA.z;                                                                           \
        a[3] = RA.w;                                                                           \
        *(float4 *)&Bs[buf][idx / 32][4 * (idx % 32)] = RB;                                     \
    }
    auto gload = [&](int64_t k0) {
        BEM_GEMM_LOAD_ONE(0, ra0, rb0)
        BEM_GEMM_LOAD_ONE(1, ra1, rb1)
        BEM_GEMM_LOAD_ONE(2, ra2, rb2)
        BEM_GEMM_LOAD_ONE(3, ra3, rb3)
    };
    auto lstore = [&](int buf) {
        BEM_GEMM_STORE_ONE(0, ra0, rb0)
        BEM_GEMM_STORE_ONE(1, ra1, rb1)
        BEM_GEMM_STORE_ONE(2, ra2, rb2)
        BEM_GEMM_STORE_ONE(3, ra3, rb3)
    };
#undef BEM_GEMM_LOAD_ONE
#undef BEM_GEMM_STORE_ONE
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
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
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

struct RankOrder {
    DevBuf<int32_t> rank, byrank, order;   // [N], [N], [T]
    std::vector<int32_t> minrank_sorted;   // [T]
    explicit RankOrder(const bem_mesh *m);
    int count_below(int r) const;
};

template <class R, bool A, bool B, bool C>
void launch_pairs(dim3 grid, hipStream_t s, bem_mesh *m, const RankOrder &ro, int n_tau, int r0,
                  DCoefT<R> cf, const DIntT<R> *itab, typename DM<R>::C *Q) {
    const R *geo;
    if constexpr (std::is_same<R, float>::value) geo = m->geo32.p;
    else geo = m->geo64.p;
    hipLaunchKernelGGL((dense_pairs_kernel<R, A, B, C>), grid, dim3(256), 0, s, geo, m->tst.p,
                       m->tobj_d.p, m->tri_d.p, m->star_ptr.p, m->star_idx.p, ro.order.p, n_tau,
                       ro.rank.p, ro.byrank.p, (int)m->T, r0, m->N, cf, itab, Q);
}

// Vertex ranks in Morton order of the coordinates (10 bits per axis over the
// bounding box, ties by index) and the triangles in ascending order of their
// smallest vertex rank; minrank_sorted[k] is that rank for order[k].
RankOrder::RankOrder(const bem_mesh *m) {
    const int64_t N = m->N, T = m->T;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < N; v++)
        for (int a = 0; a < 3; a++) {
            lo[a] = std::min(lo[a], m->P[3 * v + a]);
            hi[a] = std::max(hi[a], m->P[3 * v + a]);
        }
    std::vector<uint64_t> code(N);
    for (int64_t v = 0; v < N; v++) {
        uint64_t c = 0;
        for (int a = 0; a < 3; a++) {
            const double ext = hi[a] - lo[a];
            const double u = ext > 0 ? (m->P[3 * v + a] - lo[a]) / ext : 0.0;
            const uint64_t q = (uint64_t)std::min(1023.0, std::max(0.0, u * 1023.0));
            for (int b = 0; b < 10; b++) c |= ((q >> b) & 1u) << (3 * b + a);
        }
        code[v] = c;
    }
    std::vector<int32_t> by(N), rk(N);
    for (int64_t v = 0; v < N; v++) by[v] = (int32_t)v;
    std::stable_sort(by.begin(), by.end(), [&](int32_t a, int32_t b) { return code[a] < code[b]; });
    for (int64_t r = 0; r < N; r++) rk[by[r]] = (int32_t)r;
    std::vector<int32_t> mr(T), ord(T);
    for (int64_t t = 0; t < T; t++) {
        mr[t] = std::min(rk[m->tri[3 * t]], std::min(rk[m->tri[3 * t + 1]], rk[m->tri[3 * t + 2]]));
        ord[t] = (int32_t)t;
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return mr[a] < mr[b]; });
    minrank_sorted.resize(T);
    for (int64_t k = 0; k < T; k++) minrank_sorted[k] = mr[ord[k]];
    rank.upload(rk);
    byrank.upload(by);
    order.upload(ord);
}

// number of triangles whose smallest vertex rank is below r
int RankOrder::count_below(int r) const {
    return (int)(std::lower_bound(minrank_sorted.begin(), minrank_sorted.end(), r) -
                 minrank_sorted.begin());
}

// assembly of the operator in precision R into B ([2N][2N], row-major)
template <class R>
void assemble_into(bem_mesh *m, const NearOperator &nf, double2 k0, typename DM<R>::C *B,
                   hipStream_t s) {
    using C = typename DM<R>::C;
    const int64_t N = m->N;
    DevBuf<C> Q((size_t)m->T * JT * 12);
    const DCoefT<R> cf = make_dcoef<R>(k0, nf);
    DevBuf<R> itab;   // per-object interior parts (several objects)
    if (m->nobj > 1) {
        constexpr size_t W = sizeof(DIntT<R>) / sizeof(R);
        std::vector<R> h((size_t)m->nobj * W);
        for (int o = 0; o < m->nobj; o++) {
            const DIntT<R> c = make_dint<R>(k0, nf.k1o[o], nf.rhoo[o], nf.s1);
            std::memcpy(h.data() + (size_t)o * W, &c, sizeof(c));
        }
        itab.upload(h);
    }
    const DIntT<R> *it = (const DIntT<R> *)itab.p;
    const int code = (k0.y != 0 ? 4 : 0) | (nf.k1_plan.y != 0 ? 2 : 0) | (m->nobj > 1 ? 1 : 0);
    const RankOrder ro(m);
    for (int64_t r0 = 0; r0 < N; r0 += JT) {
        const int jt = (int)std::min<int64_t>(JT, N - r0);
        // test triangles with a vertex ranked below the tile's end
        const int n_tau = ro.count_below((int)(r0 + jt));
        if (n_tau > 0) {
            dim3 grid((unsigned)((n_tau + 255) / 256), jt);
            const int r = (int)r0;
            switch (code) {
            case 0: launch_pairs<R, false, false, false>(grid, s, m, ro, n_tau, r, cf, it, Q.p); break;
            case 1: launch_pairs<R, false, false, true>(grid, s, m, ro, n_tau, r, cf, it, Q.p); break;
            case 2: launch_pairs<R, false, true, false>(grid, s, m, ro, n_tau, r, cf, it, Q.p); break;
            case 3: launch_pairs<R, false, true, true>(grid, s, m, ro, n_tau, r, cf, it, Q.p); break;
            case 4: launch_pairs<R, true, false, false>(grid, s, m, ro, n_tau, r, cf, it, Q.p); break;
            case 5: launch_pairs<R, true, false, true>(grid, s, m, ro, n_tau, r, cf, it, Q.p); break;
            case 6: launch_pairs<R, true, true, false>(grid, s, m, ro, n_tau, r, cf, it, Q.p); break;
            default: launch_pairs<R, true, true, true>(grid, s, m, ro, n_tau, r, cf, it, Q.p); break;
            }
            BEM_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL(dense_gather_kernel<C>, dim3((unsigned)N, (jt + 255) / 256), dim3(256),
                           0, s, Q.p, m->star_ptr.p, m->star_idx.p, ro.rank.p, ro.byrank.p, N,
                           (int)r0, jt, B);
        BEM_LAUNCH_CHECK();
    }
    {
        const unsigned nt = (unsigned)((N + 31) / 32);
        hipLaunchKernelGGL(dense_mirror_kernel<C>, dim3(nt, nt, 4), dim3(256), 0, s, ro.rank.p, N,
                           B);
        BEM_LAUNCH_CHECK();
    }
    if constexpr (std::is_same<R, float>::value)
        hipLaunchKernelGGL(dense_add_near_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0,
                           s, m->nf_rowptr.p, m->nf_col.p, (const double2 *)nf.vals.p, m->nf_nnz,
                           N, B);
    else
        hipLaunchKernelGGL(dense_add_near64_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256),
                           0, s, m->nf_rowptr.p, m->nf_col.p, (const double2 *)nf.vals.p,
                           m->nf_nnz, N, B);
    BEM_LAUNCH_CHECK();
    BEM_HIP(hipStreamSynchronize(s));   // Q and the table are released on return
}

}   // namespace

int64_t dense_bytes(const bem_mesh *m, bool fp64) {
    return 4 * m->N * m->N * (int64_t)(fp64 ? sizeof(double2) : sizeof(float2));
}
int64_t dense_assembly_scratch_bytes(const bem_mesh *m, bool fp64) {
    return dense_need_bytes(m->N, m->T, fp64) - dense_bytes(m, fp64);
}
int64_t dense_need_bytes(int64_t N, int64_t T, bool fp64) {
    const int64_t c = fp64 ? sizeof(double2) : sizeof(float2);
    return 4 * N * N * c + T * (int64_t)JT * 12 * c + 2 * N * (int64_t)sizeof(float2) +
           (2 * N + T) * (int64_t)sizeof(int32_t);   // vertex ranks, triangle order
}

void dense_assemble_into(bem_mesh *m, const NearOperator &nf, double2 k0, hipStream_t s,
                         bool fp64, DenseOperator &op) {
    const int64_t n2 = 2 * m->N;
    op.n2 = n2;
    op.T = m->T;
    op.fp64 = fp64;
    Timer tm(fp64 ? "dense_assemble_fp64" : "dense_assemble", s);
    if (fp64) {
        op.B.release();
        if (op.B64.n != (size_t)(n2 * n2)) op.B64.alloc((size_t)(n2 * n2));
        assemble_into<double>(m, nf, k0, op.B64.p, s);
    } else {
        op.B64.release();
        if (op.B.n != (size_t)(n2 * n2)) op.B.alloc((size_t)(n2 * n2));
        assemble_into<float>(m, nf, k0, op.B.p, s);
    }
}

std::unique_ptr<DenseOperator> dense_assemble(bem_mesh *m, const NearOperator &nf, double2 k0,
                                              double2 k1, double rho, hipStream_t s, bool fp64) {
    (void)k1;
    (void)rho;
    auto op = std::make_unique<DenseOperator>();
    dense_assemble_into(m, nf, k0, s, fp64, *op);
    return op;
}

template <int NR>
void launch_gemv(const DenseOperator &op, const float2 *xs, double2 *y, hipStream_t s) {
    const int64_t rows = (int64_t)GV_WAVES * GV_RW;   // per workgroup
    hipLaunchKernelGGL(dense_gemv_kernel<NR>, dim3((unsigned)((op.n2 + rows - 1) / rows)),
                       dim3(64 * GV_WAVES), 0, s, op.B.p, op.n2, xs, y, op.n2);
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
    const int64_t Np = 2 * (((int64_t)R + 63) / 64) * 64, nchunks = (Kp + GKC_MIN - 1) / GKC_MIN;
    return (Kp * Np + nchunks * M * Np) * (int64_t)sizeof(float);
}

namespace {

// Split-K chunk of the MFMA product: the multiple of the K step between
// GKC_MIN and GKC whose grid fills the resident workgroup slots most evenly
// (whole waves of workgroups), longer chunks preferred at equal fill.
int gemm_kchunk(int64_t mtiles, int64_t Kp) {
    static int slots = 0;
    if (slots == 0) {
        int dev = 0, cus = 0, per = 0;
        BEM_HIP(hipGetDevice(&dev));
        BEM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        BEM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, gemm_mfma_kernel, 256, 0));
        slots = std::max(1, cus * std::max(per, 1));
    }
    int best = GKC;
    double best_fill = -1;
    for (int kc = GKC; kc >= GKC_MIN; kc -= GK) {
        const int64_t nch = (Kp + kc - 1) / kc;
        const double waves = (double)(mtiles * nch) / slots;
        const double fill = waves / std::ceil(waves);
        if (fill > best_fill + 0.01) {
            best_fill = fill;
            best = kc;
        }
    }
    return best;
}

}   // namespace

void dense_apply(const DenseOperator &op, const double2 *x, double2 *y, int R,
                 DevBuf<float2> &xs, hipStream_t s, const TuneEntry *forced) {
    if (op.fp64) {   // complex128 operator: one pass per vector
        Timer tm("dense_gemv_fp64", s);
        for (int r = 0; r < R; r++) {
            hipLaunchKernelGGL(dense_gemv64_kernel,
                               dim3((unsigned)((op.n2 + 4 * G64_RW - 1) / (4 * G64_RW))),
                               dim3(256), 0, s, op.B64.p, op.n2, x + r * op.n2, y + r * op.n2);
            BEM_LAUNCH_CHECK();
        }
        return;
    }
    const TuneEntry te = forced ? *forced : tune_lookup(op.T, R);
    if (R >= te.gemm_min) dense_gemm(op, x, y, R, s);
    else dense_gemv(op, x, y, R, xs, s, R >= te.skinny_min);
}

void dense_gemm(const DenseOperator &op, const double2 *x, double2 *y, int R, hipStream_t s) {
    const int64_t M = op.n2, K = op.n2, Kp = 2 * K;
    const int Rp = ((R + 63) / 64) * 64, Np = 2 * Rp;
    const int kchunk = gemm_kchunk(((M + GM - 1) / GM) * (Np / GN), Kp);
    const int nchunks = (int)((Kp + kchunk - 1) / kchunk);
    const size_t nx = (size_t)(Kp * Np), ny = (size_t)nchunks * M * Np;
    // the operator's workspace when no other call holds it, else our own
    DenseOperator::GemmWork &w = *op.gw;
    std::unique_lock<std::mutex> lk(w.mu, std::try_to_lock);
    DevBuf<float> own_x, own_y;
    float *Xp, *Yp;
    if (lk.owns_lock()) {
        if (w.Xp.n < nx) w.Xp.alloc(nx);
        if (w.Yp.n < ny) w.Yp.alloc(ny);
        w.held = w.Xp.bytes() + w.Yp.bytes();
        Xp = w.Xp.p;
        Yp = w.Yp.p;
    } else {
        own_x.alloc(nx);
        own_y.alloc(ny);
        Xp = own_x.p;
        Yp = own_y.p;
    }
    const int64_t prep = K * Rp;
    hipLaunchKernelGGL(gemm_xprep_kernel, dim3((unsigned)((prep + 255) / 256)), dim3(256), 0, s, x,
                       R, K, Np, Xp);
    BEM_LAUNCH_CHECK();
    {
        Timer tm("dense_gemm_mfma", s);
        hipLaunchKernelGGL(gemm_mfma_kernel,
                           dim3((unsigned)((M + GM - 1) / GM), Np / GN, nchunks), dim3(256), 0, s,
                           (const float *)op.B.p, Xp, Yp, M, Kp, Np, kchunk);
        BEM_LAUNCH_CHECK();
    }
    const int64_t red = M * R;
    hipLaunchKernelGGL(gemm_reduce_kernel, dim3((unsigned)((red + 255) / 256)), dim3(256), 0, s,
                       Yp, nchunks, M, Np, R, y);
    BEM_LAUNCH_CHECK();
    // the workspace is free again once these kernels have finished (an own
    // one is freed on return, which waits for them as well)
    if (lk.owns_lock()) BEM_HIP(hipStreamSynchronize(s));
    BEM_HIP(hipStreamSynchronize(s));   // Xp, Yp are released on return
}

namespace {
std::atomic<uint64_t> g_share_tick{0};   // last-use stamps comparable across meshes
}

int64_t DenseShare::bytes() {
    std::lock_guard<std::mutex> g(mu);
    int64_t b = 0;
    for (const auto &kv : ops) b += kv.second.op->bytes();
    return b;
}

int64_t DenseShare::idle_bytes() {
    std::lock_guard<std::mutex> g(mu);
    int64_t b = 0;
    for (const auto &kv : ops)
        if (kv.second.op.use_count() == 1) b += kv.second.op->bytes();
    return b;
}

uint64_t DenseShare::oldest_idle() {
    std::lock_guard<std::mutex> g(mu);
    uint64_t t = UINT64_MAX;
    for (const auto &kv : ops)
        if (kv.second.op.use_count() == 1) t = std::min(t, kv.second.last);
    return t;
}

int64_t DenseShare::evict_idle_lru() {
    std::shared_ptr<DenseOperator> drop;   // freed outside the lock
    {
        std::lock_guard<std::mutex> g(mu);
        auto victim = ops.end();
        for (auto it = ops.begin(); it != ops.end(); ++it)
            if (it->second.op.use_count() == 1 &&
                (victim == ops.end() || it->second.last < victim->second.last))
                victim = it;
        if (victim == ops.end()) return 0;
        drop = std::move(victim->second.op);
        ops.erase(victim);
    }
    return drop->bytes();
}

namespace {

__global__ __launch_bounds__(256) void dense_round_kernel(const double2 *__restrict__ a,
                                                          float2 *__restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256)
        b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

// into `op` (its complex64 buffer reused when it has the size)
void dense_round_into(const DenseOperator &d64, DenseOperator &o, hipStream_t s) {
    DenseOperator *op = &o;
    op->n2 = d64.n2;
    op->T = d64.T;
    op->fp64 = false;
    op->B64.release();
    const int64_t n = d64.n2 * d64.n2;
    if (op->B.n != (size_t)n) op->B.alloc((size_t)n);
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(dense_round_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d64.B64.p,
                       op->B.p, n);
    BEM_LAUNCH_CHECK();
}

std::unique_ptr<DenseOperator> dense_round(const DenseOperator &d64, hipStream_t s) {
    auto op = std::make_unique<DenseOperator>();
    dense_round_into(d64, *op, s);
    return op;
}

}   // namespace

const DenseOperator &dense_get_rounded(bem_mesh *m, double2 k0, double2 k1, double rho,
                                       hipStream_t s, int s1, const ObjMaterials *om) {
    const NearKey key = near_key(m, k0, k1, rho, s1, om);
    auto it = m->dense_rounded_cache.find(key);
    if (it != m->dense_rounded_cache.end()) return *it->second;
    const DenseOperator &d64 = dense_get(m, k0, k1, rho, s, s1, om, true);
    if (!m->dense_rounded_cache.empty()) m->dense_rounded_cache.clear();   // one at a time
    auto op = dense_round(d64, s);
    auto &ref = *op;
    m->dense_rounded_cache.emplace(key, std::move(op));
    return ref;
}

std::shared_ptr<const DenseOperator> dense_share_get(bem_mesh *m, double2 k0, double2 k1,
                                                     double rho, hipStream_t s, int s1,
                                                     const ObjMaterials *om, int kind) {
    DenseShare &sh = *m->dense_share;
    const DenseShare::Key key{near_key(m, k0, k1, rho, s1, om), kind};
    {
        std::unique_lock<std::mutex> lk(sh.mu);
        for (;;) {
            auto it = sh.ops.find(key);
            if (it != sh.ops.end()) {
                it->second.last = ++g_share_tick;
                return it->second.op;
            }
            if (!sh.building.count(key)) break;
            sh.cv.wait(lk);   // another replica assembles it
        }
        sh.building.insert(key);
    }
    // an idle operator of the same kind that the `keep` rule would drop gives
    // its buffer to the new one (no device free and allocation per new
    // wavenumber)
    std::shared_ptr<DenseOperator> op;
    {
        std::lock_guard<std::mutex> g(sh.mu);
        int idle = 0;
        auto victim = sh.ops.end();
        for (auto it = sh.ops.begin(); it != sh.ops.end(); ++it)
            if (it->second.op.use_count() == 1) {
                idle++;
                if (it->first.second == kind &&
                    (victim == sh.ops.end() || it->second.last < victim->second.last))
                    victim = it;
            }
        if (idle >= sh.keep && victim != sh.ops.end()) {
            op = std::move(victim->second.op);
            sh.ops.erase(victim);
        }
    }
    try {
        if (!op) op = std::make_shared<DenseOperator>();
        if (kind == DENSE_C64_ROUNDED) {
            // from the shared complex128 operator (held until rounded)
            const auto d64 = dense_share_get(m, k0, k1, rho, s, s1, om, DENSE_C128);
            dense_round_into(*d64, *op, s);
            BEM_HIP(hipStreamSynchronize(s));
        } else {
            const NearOperator &nf = nearfield_get(m, k0, k1, rho, s, s1, om);
            dense_assemble_into(m, nf, k0, s, kind == DENSE_C128, *op);
        }
    } catch (...) {
        std::lock_guard<std::mutex> g(sh.mu);
        sh.building.erase(key);
        sh.cv.notify_all();
        throw;
    }
    std::vector<std::shared_ptr<DenseOperator>> drop;   // freed outside the lock
    {
        std::lock_guard<std::mutex> g(sh.mu);
        sh.building.erase(key);
        sh.ops[key] = DenseShare::Entry{op, ++g_share_tick};
        // keep at most `keep` operators beside those in use
        for (;;) {
            int idle = 0;
            auto victim = sh.ops.end();
            for (auto it = sh.ops.begin(); it != sh.ops.end(); ++it)
                if (it->second.op.use_count() == 1) {   // the new one is held by `op`
                    idle++;
                    if (victim == sh.ops.end() || it->second.last < victim->second.last)
                        victim = it;
                }
            if (idle < sh.keep || victim == sh.ops.end()) break;
            drop.push_back(std::move(victim->second.op));
            sh.ops.erase(victim);
        }
        sh.cv.notify_all();
    }
    return op;
}

const DenseOperator &dense_get(bem_mesh *m, double2 k0, double2 k1, double rho, hipStream_t s,
                               int s1, const ObjMaterials *om, bool fp64) {
    const NearKey key = near_key(m, k0, k1, rho, s1, om);
    auto &cache = fp64 ? m->dense64_cache : m->dense_cache;
    auto it = cache.find(key);
    if (it != cache.end()) return *it->second;
    const NearOperator &nf = nearfield_get(m, k0, k1, rho, s, s1, om);
    // one resident dense operator per mesh unless memory allows more
    const int64_t need = dense_bytes(m, fp64) + dense_assembly_scratch_bytes(m, fp64) +
                         (int64_t)(1ll << 30);
    size_t free_b = 0, total_b = 0;
    BEM_HIP(hipMemGetInfo(&free_b, &total_b));
    while ((!m->dense_cache.empty() || !m->dense64_cache.empty()) && (int64_t)free_b < need) {
        auto &victim = m->dense64_cache.empty() ? m->dense_cache : m->dense64_cache;
        victim.erase(victim.begin());
        BEM_HIP(hipMemGetInfo(&free_b, &total_b));
    }
    if ((int64_t)free_b < need)
        fail(BEM_E_NOMEM, "dense operator of " + std::to_string(dense_bytes(m, fp64)) +
                              " bytes does not fit in device memory");
    auto op = dense_assemble(m, nf, k0, k1, rho, s, fp64);
    auto &ref = *op;
    cache.emplace(key, std::move(op));
    return ref;
}

}   // namespace bem

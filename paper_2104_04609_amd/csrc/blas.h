// Complex FP64 vector kernels used by GMRES (deterministic reductions).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bem {

// h[i] = <V_i, w> = sum_k conj(V[i][k]) w[k], i < m (V row-major, stride ld)
void blas_block_dot(const double2 *V, int64_t ld, int m, const double2 *w, int64_t n,
                    double2 *h, hipStream_t s);
// w += sign * sum_{i<m} h[i] V_i
void blas_block_axpy(const double2 *V, int64_t ld, const double2 *h, int m, double sign,
                     double2 *w, int64_t n, hipStream_t s);
// v /= sqrt(Re nrm2[0]), in place
void blas_normalize(double2 *v, const double2 *nrm2, int64_t n, hipStream_t s);
// out = a x + b y  (y may be NULL; out may alias x or y)
void blas_axpby(double2 a, const double2 *x, double2 b, const double2 *y, double2 *out,
                int64_t n, hipStream_t s);

// The same for A <= BLAS_MAX_BATCH independent systems in one launch each
// (system a: basis V[a] with stride ld, vector w[a], output h[a]; the
// per-system arithmetic and its order do not depend on A).  The dot products
// are summed per chunk of BLAS_DOT_CHUNK entries (fixed-order tree), then the
// chunks in order; `part` holds A * m * blas_dot_chunks(n) entries.
constexpr int BLAS_MAX_BATCH = 16;
constexpr int BLAS_DOT_CHUNK = 2048;
struct CVecs {
    const double2 *p[BLAS_MAX_BATCH];
};
struct Vecs {
    double2 *p[BLAS_MAX_BATCH];
};
inline int64_t blas_dot_chunks(int64_t n) { return (n + BLAS_DOT_CHUNK - 1) / BLAS_DOT_CHUNK; }
void blas_block_dot_batch(const CVecs &V, int64_t ld, int m, const CVecs &w, int64_t n,
                          const Vecs &h, int A, double2 *part, hipStream_t s);
void blas_block_axpy_batch(const CVecs &V, int64_t ld, const CVecs &h, int m, double sign,
                           const Vecs &w, int64_t n, int A, hipStream_t s);
void blas_normalize_batch(const Vecs &v, const CVecs &nrm2, int64_t n, int A, hipStream_t s);
// dst[a] = src[a] (n entries each)
void blas_copy_batch(const Vecs &dst, const CVecs &src, int64_t n, int A, hipStream_t s);

// sub[r] = [x_r[idx]; x_r[N + idx]] for R vectors (x [R][2N], sub [R][2 nm])
void gather_halves(const double2 *x, const int32_t *idx, int64_t N, int64_t nm, int R,
                   double2 *sub, hipStream_t s);
// the inverse: x_r[idx] = sub_r[:nm], x_r[N + idx] = sub_r[nm:]
void scatter_halves(const double2 *sub, const int32_t *idx, int64_t N, int64_t nm, int R,
                    double2 *x, hipStream_t s);

}   // namespace bem

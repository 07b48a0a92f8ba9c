// Near-field operator of the permuted PMCHWT matvec (FP64, built once per
// (k_ext, k_int, rho, s1) and kept on the device).
//
// For every ordered triangle pair (tau, sigma) sharing at least one vertex the
// four combined 3x3 blocks
//   B11 = V_0 + rho V_1,  B12 = -(K_0 + K_1),  B21 = K'_0 + K'_1,
//   B22 = D_0 + D_1 / rho          (Sec. 2.7; operators of Sec. 2.2)
// are integrated with the singular rule of the pair's class (coincident,
// common edge, common vertex); the matrix-free pair kernel skips exactly these
// pairs.  The blocks are summed into a vertex-by-vertex CSR matrix in a fixed
// order.  The interior terms of a pair use its object's material.  With s1 =
// -1 the interior terms enter with the opposite sign and the
// coincident pairs add the local P1 mass matrix |tau| (1 + delta_ab) / 12 to
// B12 and B21: the Mueller operator I + A_0 - A^_1 of Sec. 2.2 on the
// permuted unknowns, whose identity pairs each trace row with its own trace.
#include <cmath>

#include "bem_internal.h"

namespace bem {

namespace {

struct NearCoef {
    double2 k0;
    double s1;   // +1 PMCHWT, -1 Mueller
};

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// e^{i k r} / (4 pi r) and (i k r - 1) e^{i k r} / (4 pi r^3)
__device__ inline void green(double2 k, double r, double2 &G, double2 &F) {
    double s, c;
    sincos(k.x * r, &s, &c);
    double mag = exp(-k.y * r) * (0.079577471545947667884441881686257 / r);
    G = make_double2(c * mag, s * mag);
    double2 t = make_double2(-1.0 - k.y * r, k.x * r);   // i k r - 1
    F = cmul(G, t);
    double ir2 = 1.0 / (r * r);
    F.x *= ir2;
    F.y *= ir2;
}

constexpr int NACC = 74;   // 4 x 9 complex blocks (B22 normal part) + 1 complex

// One wave (64 lanes) per ordered pair.
__global__ __launch_bounds__(64) void near_pairs_kernel(
    const int32_t *__restrict__ pairs, int64_t n_pairs, const double *__restrict__ P,
    const int32_t *__restrict__ tri, const double *__restrict__ tst,
    const double *__restrict__ geo, const double *__restrict__ tab, int off0, int off1,
    int off2, int off3, NearCoef cf, const int32_t *__restrict__ tobj,
    const double *__restrict__ omat, double2 *__restrict__ blocks) {
    const int64_t p = blockIdx.x;
    if (p >= n_pairs) return;
    const int lane = threadIdx.x;
    const int t = pairs[4 * p], s = pairs[4 * p + 1], cls = pairs[4 * p + 2],
              perm = pairs[4 * p + 3];
    int px[3], py[3];
    for (int r = 0; r < 3; r++) {
        px[r] = (perm >> (2 * r)) & 3;
        py[r] = (perm >> (6 + 2 * r)) & 3;
    }
    double vt[3][3], vs[3][3];
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) {
            vt[a][c] = P[3 * tri[3 * t + a] + c];
            vs[a][c] = P[3 * tri[3 * s + a] + c];
        }
    const double at = tst[TST_STRIDE * t], as = tst[TST_STRIDE * s];
    const double *nt = geo + GEO_STRIDE * t + 18, *ns = geo + GEO_STRIDE * s + 18;
    const double nn = nt[0] * ns[0] + nt[1] * ns[1] + nt[2] * ns[2];

    const int rb = cls == 0 ? off0 : (cls == 1 ? off1 : off2);
    const int re = cls == 0 ? off1 : (cls == 1 ? off2 : off3);
    const int nss = re - rb;

    double acc[NACC];
#pragma unroll
    for (int i = 0; i < NACC; i++) acc[i] = 0.0;
    const double k0sq_r = cf.k0.x * cf.k0.x - cf.k0.y * cf.k0.y, k0sq_i = 2 * cf.k0.x * cf.k0.y;
    // interior material of the pair's object (a pair sharing a vertex lies
    // within one object): omat[object] = (Re k_1, Im k_1, rho)
    const int ob = tobj[t];
    const double2 k1 = make_double2(omat[3 * ob], omat[3 * ob + 1]);
    const double rho = omat[3 * ob + 2];
    const double k1sq_r = cf.s1 * (k1.x * k1.x - k1.y * k1.y) / rho,
                 k1sq_i = cf.s1 * 2 * k1.x * k1.y / rho;
    const double rho1 = cf.s1 * rho, irho1 = cf.s1 / rho;

    for (int q = lane; q < nss; q += 64) {
        double lx[3], ly[3];
        const double *row = tab + 5 * (int64_t)(rb + q);
        const double bx[3] = {1.0 - row[0], row[0] - row[1], row[1]};
        const double by[3] = {1.0 - row[2], row[2] - row[3], row[3]};
        for (int r = 0; r < 3; r++) {
            lx[px[r]] = bx[r];
            ly[py[r]] = by[r];
        }
        const double w = 4.0 * at * as * row[4];
        double d[3];
        for (int c = 0; c < 3; c++) {
            double xc = lx[0] * vt[0][c] + lx[1] * vt[1][c] + lx[2] * vt[2][c];
            double yc = ly[0] * vs[0][c] + ly[1] * vs[1][c] + ly[2] * vs[2][c];
            d[c] = xc - yc;   // x - y
        }
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double2 G0, F0, G1, F1;
        green(cf.k0, r, G0, F0);
        green(k1, r, G1, F1);
        double2 GV = make_double2(G0.x + rho1 * G1.x, G0.y + rho1 * G1.y);
        double2 GW = make_double2(G0.x + irho1 * G1.x, G0.y + irho1 * G1.y);
        double2 GN = make_double2(k0sq_r * G0.x - k0sq_i * G0.y + k1sq_r * G1.x - k1sq_i * G1.y,
                                  k0sq_r * G0.y + k0sq_i * G0.x + k1sq_r * G1.y + k1sq_i * G1.x);
        double2 FK = make_double2(F0.x + cf.s1 * F1.x, F0.y + cf.s1 * F1.y);
        double dny = -(d[0] * ns[0] + d[1] * ns[1] + d[2] * ns[2]);   // (y-x).n_y
        double dnx = d[0] * nt[0] + d[1] * nt[1] + d[2] * nt[2];      // (x-y).n_x
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                double pp = w * lx[a] * ly[b];
                int e = 2 * (3 * a + b);
                acc[e] += GV.x * pp;
                acc[e + 1] += GV.y * pp;
                acc[18 + e] -= FK.x * dny * pp;
                acc[18 + e + 1] -= FK.y * dny * pp;
                acc[36 + e] += FK.x * dnx * pp;
                acc[36 + e + 1] += FK.y * dnx * pp;
                acc[54 + e] -= GN.x * nn * pp;
                acc[54 + e + 1] -= GN.y * nn * pp;
            }
        acc[72] += GW.x * w;
        acc[73] += GW.y * w;
    }
    // wave reduction (fixed butterfly order)
#pragma unroll
    for (int i = 0; i < NACC; i++) {
        double v = acc[i];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        acc[i] = v;
    }
    if (lane == 0) {
#pragma unroll
        for (int e = 0; e < 36; e++) {
            const int blk = e / 9, ab = e % 9, a = ab / 3, b = ab % 3;
            double2 v = make_double2(acc[18 * blk + 2 * ab], acc[18 * blk + 2 * ab + 1]);
            if (blk == 3) {
                const double *ca = tst + TST_STRIDE * t + 1 + 3 * a;
                const double *cb = tst + TST_STRIDE * s + 1 + 3 * b;
                const double cc = ca[0] * cb[0] + ca[1] * cb[1] + ca[2] * cb[2];
                v.x += cc * acc[72];
                v.y += cc * acc[73];
            }
            if (cf.s1 < 0 && t == s && (blk == 1 || blk == 2))
                v.x += at * (a == b ? 2.0 : 1.0) / 12.0;   // Mueller identity: P1 mass
            blocks[36 * p + e] = v;
        }
    }
}

// CSR values: C[blk][e] = sum over the entry's contributions (fixed order).
__global__ __launch_bounds__(256) void near_csr_kernel(
    const int32_t *__restrict__ cptr, const int32_t *__restrict__ contrib, int64_t nnz,
    const double2 *__restrict__ blocks, double2 *__restrict__ vals) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    double2 acc[4];
    for (int b = 0; b < 4; b++) acc[b] = make_double2(0.0, 0.0);
    for (int c = cptr[e]; c < cptr[e + 1]; c++) {
        int code = contrib[c];
        int64_t p = code / 9;
        int ab = code - 9 * (int)p;
        for (int b = 0; b < 4; b++) {
            double2 v = blocks[36 * p + 9 * b + ab];
            acc[b].x += v.x;
            acc[b].y += v.y;
        }
    }
    for (int b = 0; b < 4; b++) vals[b * nnz + e] = acc[b];
}

}   // namespace

NearKey near_key(const bem_mesh *m, double2 k0, double2 k1, double rho, int s1,
                 const ObjMaterials *om) {
    s1 = s1 < 0 ? -1 : 1;
    NearKey key{k0.x, k0.y, k1.x, k1.y, rho, s1, {}};
    if (om) {
        bool same = true;
        for (int o = 1; o < m->nobj; o++)
            same = same && om->k[o].x == om->k[0].x && om->k[o].y == om->k[0].y &&
                   om->rho[o] == om->rho[0];
        key.k1r = om->k[0].x;
        key.k1i = om->k[0].y;
        key.rho = om->rho[0];
        if (!same)
            for (int o = 0; o < m->nobj; o++) {
                key.om.push_back(om->k[o].x);
                key.om.push_back(om->k[o].y);
                key.om.push_back(om->rho[o]);
            }
    }
    return key;
}

std::unique_ptr<NearOperator> nearfield_build(bem_mesh *m, double2 k0, double2 k1,
                                              double rho, hipStream_t s, int s1,
                                              const ObjMaterials *om) {
    auto op = std::make_unique<NearOperator>();
    op->s1 = s1 < 0 ? -1 : 1;
    op->k1o.assign(m->nobj, k1);
    op->rhoo.assign(m->nobj, rho);
    if (om) {
        op->k1o = om->k;
        op->rhoo = om->rho;
    }
    std::vector<double> mat(3 * (size_t)m->nobj);
    bool complex_k = false;
    op->k1_plan = op->k1o[0];
    for (int o = 0; o < m->nobj; o++) {
        mat[3 * o] = op->k1o[o].x;
        mat[3 * o + 1] = op->k1o[o].y;
        mat[3 * o + 2] = op->rhoo[o];
        complex_k = complex_k || op->k1o[o].y != 0.0;
        if (std::fabs(op->k1o[o].x) > std::fabs(op->k1_plan.x)) op->k1_plan = op->k1o[o];
    }
    if (complex_k && op->k1_plan.y == 0.0) op->k1_plan.y = 1.0;   // any complex k_m: complex variant
    op->vals.alloc(4 * (size_t)m->nf_nnz * 2);
    DevBuf<double> Pd, matd;
    std::vector<double> Ph(m->P);
    Pd.upload(Ph);
    matd.upload(mat);
    DevBuf<double2> blocks(36 * (size_t)m->n_near);
    NearCoef cf{k0, (double)op->s1};
    {
        Timer tm("nearfield_build", s);
        hipLaunchKernelGGL(near_pairs_kernel, dim3((unsigned)m->n_near), dim3(64), 0, s,
                           m->near_pairs.p, m->n_near, Pd.p, m->tri_d.p, m->tst.p,
                           m->geo64.p, m->ss_tab.p, m->ss_off[0], m->ss_off[1],
                           m->ss_off[2], m->ss_off[3], cf, m->tobj_d.p, matd.p, blocks.p);
        BEM_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(near_csr_kernel, dim3((unsigned)((m->nf_nnz + 255) / 256)), dim3(256),
                       0, s, m->nf_cptr.p, m->nf_contrib.p, m->nf_nnz, blocks.p,
                       (double2 *)op->vals.p);
    BEM_LAUNCH_CHECK();
    BEM_HIP(hipStreamSynchronize(s));
    return op;
}

const NearOperator &nearfield_get(bem_mesh *m, double2 k0, double2 k1, double rho,
                                  hipStream_t s, int s1, const ObjMaterials *om) {
    const NearKey key = near_key(m, k0, k1, rho, s1, om);
    auto it = m->near_cache.find(key);
    if (it != m->near_cache.end()) return *it->second;
    if (m->near_cache.size() >= 8) m->near_cache.erase(m->near_cache.begin());
    auto op = nearfield_build(m, k0, make_double2(key.k1r, key.k1i), key.rho, s, key.s1,
                              key.om.empty() ? nullptr : om);
    auto &ref = *op;
    m->near_cache.emplace(key, std::move(op));
    return ref;
}

}   // namespace bem

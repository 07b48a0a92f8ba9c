// Mesh state: validation of a closed, outward-oriented surface (Sec. 2.1:
// bounded objects with outward unit normals), P1 geometry (Sec. 2.3), the
// adjacency classes that decide which triangle pairs need singular quadrature,
// and the device-resident records used by the kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "bem_internal.h"

namespace bem {

namespace {

void cross(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

uint64_t edge_key(int32_t a, int32_t b) { return ((uint64_t)(uint32_t)a << 32) | (uint32_t)b; }

}   // namespace

void mesh_build(bem_mesh *m, const double *P, int64_t N, const int32_t *tri,
                int64_t T, const int32_t *obj) {
    if (!P || !tri || N < 4 || T < 4) fail(BEM_E_INVAL, "mesh needs >= 4 vertices and triangles");
    // vertex ids travel through the FP32 pair kernel as floats: N < 2^24
    if (N >= (1 << 24) || T >= (1 << 25)) fail(BEM_E_INVAL, "mesh too large");
    m->N = N;
    m->T = T;
    m->P.assign(P, P + 3 * N);
    m->tri.assign(tri, tri + 3 * T);
    m->tobj.assign(T, 0);
    int nobj = 1;
    if (obj) {
        int mx = 0;
        for (int64_t t = 0; t < T; t++) {
            if (obj[t] < 0) fail(BEM_E_INVAL, "negative object id");
            mx = std::max(mx, obj[t]);
            m->tobj[t] = obj[t];
        }
        nobj = mx + 1;
    }
    m->nobj = nobj;
    for (int64_t i = 0; i < 3 * T; i++)
        if (tri[i] < 0 || tri[i] >= N) fail(BEM_E_INVAL, "triangle index out of range");
    for (int64_t i = 0; i < 3 * N; i++)
        if (!std::isfinite(P[i])) fail(BEM_E_INVAL, "non-finite vertex coordinate");

    // bounding box, centre
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = 0; v < N; v++)
        for (int c = 0; c < 3; c++) {
            lo[c] = std::min(lo[c], P[3 * v + c]);
            hi[c] = std::max(hi[c], P[3 * v + c]);
        }
    double diag2 = 0;
    for (int c = 0; c < 3; c++) {
        m->centre[c] = 0.5 * (lo[c] + hi[c]);
        diag2 += (hi[c] - lo[c]) * (hi[c] - lo[c]);
    }
    m->diameter = std::sqrt(diag2);

    // vertex ownership by object
    m->vobj.assign(N, -1);
    std::vector<int> used(N, 0);
    for (int64_t t = 0; t < T; t++)
        for (int a = 0; a < 3; a++) {
            int v = tri[3 * t + a];
            used[v] = 1;
            if (m->vobj[v] < 0) m->vobj[v] = m->tobj[t];
            else if (m->vobj[v] != m->tobj[t])
                fail(BEM_E_BAD_MESH, "vertex " + std::to_string(v) + " shared by two objects");
        }
    for (int64_t v = 0; v < N; v++)
        if (!used[v]) fail(BEM_E_BAD_MESH, "vertex " + std::to_string(v) + " is not used");
    for (int64_t v = 1; v < N; v++)
        if (m->vobj[v] < m->vobj[v - 1])
            fail(BEM_E_BAD_MESH, "vertices of each object must be contiguous and ordered by object id");

    // geometry
    m->area.assign(T, 0);
    m->normal.assign(3 * T, 0);
    m->curl.assign(9 * T, 0);
    for (int64_t t = 0; t < T; t++) {
        const double *v[3];
        for (int a = 0; a < 3; a++) v[a] = &P[3 * tri[3 * t + a]];
        double e1[3], e2[3], n[3];
        for (int c = 0; c < 3; c++) {
            e1[c] = v[1][c] - v[0][c];
            e2[c] = v[2][c] - v[0][c];
        }
        cross(e1, e2, n);
        double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (!(0.5 * len > 1e-14 * diag2))
            fail(BEM_E_BAD_MESH, "degenerate triangle " + std::to_string(t));
        m->area[t] = 0.5 * len;
        for (int c = 0; c < 3; c++) m->normal[3 * t + c] = n[c] / len;
        for (int a = 0; a < 3; a++) {
            double e[3], g[3], cu[3];
            for (int c = 0; c < 3; c++) e[c] = v[(a + 2) % 3][c] - v[(a + 1) % 3][c];
            cross(&m->normal[3 * t], e, g);   // grad phi_a * 2|tau|
            for (int c = 0; c < 3; c++) g[c] /= 2.0 * m->area[t];
            cross(&m->normal[3 * t], g, cu);  // curl phi_a = n x grad phi_a
            for (int c = 0; c < 3; c++) m->curl[9 * t + 3 * a + c] = cu[c];
        }
    }

    // closed, manifold, consistently oriented: every directed edge once and
    // its reverse once
    std::unordered_map<uint64_t, int> dir;
    dir.reserve(6 * T);
    for (int64_t t = 0; t < T; t++)
        for (int a = 0; a < 3; a++) {
            uint64_t k = edge_key(tri[3 * t + a], tri[3 * t + (a + 1) % 3]);
            if (++dir[k] > 1)
                fail(BEM_E_BAD_MESH, "directed edge used twice (non-manifold or inconsistent orientation)");
        }
    for (const auto &kv : dir) {
        int32_t a = (int32_t)(kv.first >> 32), b = (int32_t)(kv.first & 0xffffffffu);
        if (!dir.count(edge_key(b, a)))
            fail(BEM_E_BAD_MESH, "open edge " + std::to_string(a) + "-" + std::to_string(b));
    }
    // outward orientation and radius per object
    std::vector<double> vol(nobj, 0.0);
    for (int64_t t = 0; t < T; t++) {
        const double *v0 = &P[3 * tri[3 * t]], *v1 = &P[3 * tri[3 * t + 1]],
                     *v2 = &P[3 * tri[3 * t + 2]];
        double c[3];
        cross(v1, v2, c);
        vol[m->tobj[t]] += (v0[0] * c[0] + v0[1] * c[1] + v0[2] * c[2]) / 6.0;
    }
    m->obj_radius.assign(nobj, 0.0);
    for (int o = 0; o < nobj; o++) {
        if (!(vol[o] > 0))
            fail(BEM_E_BAD_MESH, "object " + std::to_string(o) +
                                     " has non-positive signed volume (inward normals or empty)");
        double cen[3] = {0, 0, 0};
        int64_t cnt = 0;
        for (int64_t v = 0; v < N; v++)
            if (m->vobj[v] == o) {
                for (int c = 0; c < 3; c++) cen[c] += P[3 * v + c];
                cnt++;
            }
        for (int c = 0; c < 3; c++) cen[c] /= (double)cnt;
        double r = 0;
        for (int64_t v = 0; v < N; v++)
            if (m->vobj[v] == o) {
                double d2 = 0;
                for (int c = 0; c < 3; c++) d2 += (P[3 * v + c] - cen[c]) * (P[3 * v + c] - cen[c]);
                r = std::max(r, std::sqrt(d2));
            }
        m->obj_radius[o] = r;
    }

    // device geometry records
    const Rules &R = rules();
    std::vector<double> g64(GEO_STRIDE * T);
    std::vector<float> g32(GEO_STRIDE * T);
    std::vector<double> tst(TST_STRIDE * T);
    for (int64_t t = 0; t < T; t++) {
        const double *v[3];
        for (int a = 0; a < 3; a++) v[a] = &P[3 * tri[3 * t + a]];
        for (int q = 0; q < 6; q++)
            for (int c = 0; c < 3; c++) {
                double x = R.reg_bary[q][0] * v[0][c] + R.reg_bary[q][1] * v[1][c] +
                           R.reg_bary[q][2] * v[2][c];
                g64[GEO_STRIDE * t + 3 * q + c] = x;
                g32[GEO_STRIDE * t + 3 * q + c] = (float)(x - m->centre[c]);
            }
        double c64 = 0, c32 = 0;
        for (int c = 0; c < 3; c++) {
            double n = m->normal[3 * t + c];
            g64[GEO_STRIDE * t + 18 + c] = n;
            g32[GEO_STRIDE * t + 18 + c] = (float)n;
            c64 += n * v[0][c];
            c32 += n * (v[0][c] - m->centre[c]);
        }
        g64[GEO_STRIDE * t + 21] = c64;
        g32[GEO_STRIDE * t + 21] = (float)c32;
        tst[TST_STRIDE * t] = m->area[t];
        for (int i = 0; i < 9; i++) tst[TST_STRIDE * t + 1 + i] = m->curl[9 * t + i];
    }
    m->geo64.upload(g64);
    m->geo32.upload(g32);
    m->tst.upload(tst);
    m->tobj_d.upload(m->tobj);
    m->tri_d.upload(m->tri);

    // vertex star: (tri*3 + a) in ascending order
    std::vector<int32_t> sptr(N + 1, 0), sidx(3 * T);
    for (int64_t i = 0; i < 3 * T; i++) sptr[tri[i] + 1]++;
    for (int64_t v = 0; v < N; v++) sptr[v + 1] += sptr[v];
    {
        std::vector<int32_t> fill(sptr.begin(), sptr.end() - 1);
        for (int64_t i = 0; i < 3 * T; i++) sidx[fill[tri[i]]++] = (int32_t)i;
    }
    m->star_ptr.upload(sptr);
    m->star_idx.upload(sidx);

    // near pairs: ordered (tau, sigma) sharing >= 1 vertex, tau-major, sigma
    // ascending; class 0 coincident, 1 common edge, 2 common vertex
    std::vector<int32_t> pairs;
    std::vector<int32_t> cand;
    for (int64_t t = 0; t < T; t++) {
        cand.clear();
        for (int a = 0; a < 3; a++) {
            int v = tri[3 * t + a];
            for (int e = sptr[v]; e < sptr[v + 1]; e++) cand.push_back(sidx[e] / 3);
        }
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        for (int s : cand) {
            int px[3] = {0, 1, 2}, py[3] = {0, 1, 2}, cls;
            int shared[3], ns = 0;
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                    if (tri[3 * t + a] == tri[3 * s + b]) shared[ns++] = tri[3 * t + a];
            if (s == t) {
                cls = 0;
            } else if (ns == 2) {
                cls = 1;
                int A = std::min(shared[0], shared[1]), B = std::max(shared[0], shared[1]);
                for (int a = 0; a < 3; a++) {
                    int vt = tri[3 * t + a], vs = tri[3 * s + a];
                    if (vt == A) px[0] = a; else if (vt == B) px[1] = a; else px[2] = a;
                    if (vs == A) py[0] = a; else if (vs == B) py[1] = a; else py[2] = a;
                }
            } else if (ns == 1) {
                cls = 2;
                for (int a = 0; a < 3; a++) {
                    if (tri[3 * t + a] == shared[0])
                        for (int r = 0; r < 3; r++) px[r] = (a + r) % 3;
                    if (tri[3 * s + a] == shared[0])
                        for (int r = 0; r < 3; r++) py[r] = (a + r) % 3;
                }
            } else {
                fail(BEM_E_BAD_MESH, "distinct triangles share all three vertices");
            }
            int perm = px[0] | (px[1] << 2) | (px[2] << 4) | (py[0] << 6) |
                       (py[1] << 8) | (py[2] << 10);
            pairs.push_back((int32_t)t);
            pairs.push_back(s);
            pairs.push_back(cls);
            pairs.push_back(perm);
        }
    }
    m->n_near = (int64_t)pairs.size() / 4;
    m->near_pairs.upload(pairs);

    // near-field CSR pattern (vertex rows x vertex columns) and, per entry,
    // the contributing (pair, a, b) in ascending order
    std::vector<std::vector<int32_t>> rows(N);
    for (int64_t p = 0; p < m->n_near; p++) {
        int t = pairs[4 * p], s = pairs[4 * p + 1];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) rows[tri[3 * t + a]].push_back(tri[3 * s + b]);
    }
    std::vector<int32_t> rptr(N + 1, 0), col;
    for (int64_t i = 0; i < N; i++) {
        auto &r = rows[i];
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        rptr[i + 1] = rptr[i] + (int32_t)r.size();
    }
    col.reserve(rptr[N]);
    for (int64_t i = 0; i < N; i++) col.insert(col.end(), rows[i].begin(), rows[i].end());
    rows.clear();
    rows.shrink_to_fit();
    m->nf_nnz = rptr[N];
    auto find = [&](int i, int j) {
        auto it = std::lower_bound(col.begin() + rptr[i], col.begin() + rptr[i + 1], j);
        return (int32_t)(it - col.begin());
    };
    std::vector<int32_t> cptr(m->nf_nnz + 1, 0);
    for (int64_t p = 0; p < m->n_near; p++) {
        int t = pairs[4 * p], s = pairs[4 * p + 1];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) cptr[find(tri[3 * t + a], tri[3 * s + b]) + 1]++;
    }
    for (int64_t e = 0; e < m->nf_nnz; e++) cptr[e + 1] += cptr[e];
    std::vector<int32_t> contrib(cptr[m->nf_nnz]);
    {
        std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
        for (int64_t p = 0; p < m->n_near; p++) {
            int t = pairs[4 * p], s = pairs[4 * p + 1];
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                    contrib[fill[find(tri[3 * t + a], tri[3 * s + b])]++] =
                        (int32_t)(9 * p + 3 * a + b);
        }
    }
    m->nf_rowptr.upload(rptr);
    m->nf_col.upload(col);
    m->nf_cptr.upload(cptr);
    m->nf_contrib.upload(contrib);

    // singular rules, concatenated
    std::vector<double> tab;
    for (int c = 0; c < 3; c++) {
        m->ss_off[c] = (int)(tab.size() / 5);
        tab.insert(tab.end(), R.ss[c].begin(), R.ss[c].end());
    }
    m->ss_off[3] = (int)(tab.size() / 5);
    m->ss_tab.upload(tab);
}

void mesh_parts(bem_mesh *m) {
    if (!m->parts.empty()) return;
    std::vector<int64_t> local(m->N, -1);
    for (int o = 0; o < m->nobj; o++) {
        std::vector<int32_t> vid;
        for (int64_t v = 0; v < m->N; v++)
            if (m->vobj[v] == o) {
                local[v] = (int64_t)vid.size();
                vid.push_back((int32_t)v);
            }
        std::vector<double> P(3 * vid.size());
        for (size_t i = 0; i < vid.size(); i++)
            for (int c = 0; c < 3; c++) P[3 * i + c] = m->P[3 * (size_t)vid[i] + c];
        std::vector<int32_t> tri;
        for (int64_t t = 0; t < m->T; t++)
            if (m->tobj[t] == o)
                for (int a = 0; a < 3; a++) tri.push_back((int32_t)local[m->tri[3 * t + a]]);
        auto pm = std::make_unique<bem_mesh>();
        mesh_build(pm.get(), P.data(), (int64_t)vid.size(), tri.data(), (int64_t)tri.size() / 3,
                   nullptr);
        m->parts.push_back(std::move(pm));
        DevBuf<int32_t> d;
        d.upload(vid);
        m->part_vidx.push_back(std::move(d));
    }
}

}   // namespace bem

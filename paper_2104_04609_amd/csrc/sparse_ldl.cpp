// Sparse complex-symmetric LDL^T: nested dissection, symbolic analysis,
// left-looking numeric factorisation, level schedules for the GPU solves.
#include "sparse_ldl.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace bem {

namespace {

// Returns the height of the subtree rooted at this call (-1 if empty).
int dissect(std::vector<int32_t> &vs, const std::vector<int32_t> &ptr,
            const std::vector<int32_t> &col, const std::vector<double> &xyz,
            std::vector<int32_t> &side, NdOrder &nd, int leaf) {
    if (vs.empty()) return -1;
    const int first = (int)nd.bheight.size();   // blocks of this call start here
    auto emit = [&](const std::vector<int32_t> &blk, int h) {
        nd.bstart.push_back((int32_t)nd.order.size());
        nd.bheight.push_back(h);
        nd.bfirst.push_back(first);
        nd.order.insert(nd.order.end(), blk.begin(), blk.end());
    };
    if ((int)vs.size() <= leaf) {
        emit(vs, 0);
        return 0;
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int v : vs)
        for (int c = 0; c < 3; c++) {
            lo[c] = std::min(lo[c], xyz[3 * v + c]);
            hi[c] = std::max(hi[c], xyz[3 * v + c]);
        }
    int ax = 0;
    for (int c = 1; c < 3; c++)
        if (hi[c] - lo[c] > hi[ax] - lo[ax]) ax = c;
    size_t mid = vs.size() / 2;
    std::nth_element(vs.begin(), vs.begin() + mid, vs.end(), [&](int a, int b) {
        double xa = xyz[3 * a + ax], xb = xyz[3 * b + ax];
        return xa < xb || (xa == xb && a < b);
    });
    // side: 1 = part A, 2 = part B (only vertices of this subset are marked)
    for (size_t i = 0; i < vs.size(); i++) side[vs[i]] = i < mid ? 1 : 2;
    std::vector<int32_t> A, B, S;
    for (size_t i = 0; i < vs.size(); i++) {
        int v = vs[i];
        if (side[v] == 1) {
            A.push_back(v);
            continue;
        }
        bool sep = false;
        for (int e = ptr[v]; e < ptr[v + 1] && !sep; e++) sep = side[col[e]] == 1;
        (sep ? S : B).push_back(v);
    }
    for (int v : vs) side[v] = 0;
    if (A.empty() || B.empty()) {   // cannot split further (degenerate geometry)
        emit(vs, 0);
        return 0;
    }
    std::sort(A.begin(), A.end());
    std::sort(B.begin(), B.end());
    std::sort(S.begin(), S.end());
    const int ha = dissect(A, ptr, col, xyz, side, nd, leaf);
    const int hb = dissect(B, ptr, col, xyz, side, nd, leaf);
    const int h = std::max(ha, hb) + 1;
    if (S.empty()) return h - 1;
    emit(S, h);
    return h;
}

}   // namespace

NdOrder nested_dissection(int n, const std::vector<int32_t> &ptr, const std::vector<int32_t> &col,
                          const std::vector<double> &xyz, const std::vector<int32_t> &group,
                          int leaf) {
    NdOrder nd;
    std::vector<int32_t> side(n, 0);
    nd.order.reserve(n);
    int ng = 0;
    for (int v = 0; v < n; v++) ng = std::max(ng, group[v] + 1);
    for (int g = 0; g < ng; g++) {
        std::vector<int32_t> vs;
        for (int v = 0; v < n; v++)
            if (group[v] == g) vs.push_back(v);
        dissect(vs, ptr, col, xyz, side, nd, leaf);
    }
    nd.bstart.push_back((int32_t)nd.order.size());
    return nd;
}

LdlSymbolic ldl_symbolic(int n, const std::vector<int32_t> &ptr,
                         const std::vector<int32_t> &col, const NdOrder &nd) {
    LdlSymbolic S;
    S.n = n;
    S.perm = nd.order;
    const std::vector<int32_t> &perm = nd.order;
    S.iperm.assign(n, 0);
    for (int i = 0; i < n; i++) S.iperm[perm[i]] = i;

    // permuted lower triangle (CSC by new column), with source positions
    std::vector<std::vector<std::pair<int32_t, int32_t>>> cols(n);
    for (int r = 0; r < n; r++)
        for (int e = ptr[r]; e < ptr[r + 1]; e++) {
            int i = S.iperm[r], j = S.iperm[col[e]];
            if (i >= j) cols[j].push_back({i, e});
        }
    S.Ap.assign(n + 1, 0);
    for (int j = 0; j < n; j++) {
        std::sort(cols[j].begin(), cols[j].end());
        S.Ap[j + 1] = S.Ap[j] + (int32_t)cols[j].size();
    }
    S.Ai.reserve(S.Ap[n]);
    S.Asrc.reserve(S.Ap[n]);
    for (int j = 0; j < n; j++)
        for (auto &pe : cols[j]) {
            S.Ai.push_back(pe.first);
            S.Asrc.push_back(pe.second);
        }

    // elimination tree (Liu): process rows i; entries (i, k), k < i
    // rows of the lower triangle = columns of the upper: build row lists
    std::vector<std::vector<int32_t>> rowk(n);
    for (int j = 0; j < n; j++)
        for (int p = S.Ap[j]; p < S.Ap[j + 1]; p++)
            if (S.Ai[p] > j) rowk[S.Ai[p]].push_back(j);
    S.parent.assign(n, -1);
    std::vector<int32_t> anc(n, -1);
    for (int i = 0; i < n; i++)
        for (int k : rowk[i]) {
            int r = k;
            while (r != -1 && r < i) {
                int nx = anc[r];
                anc[r] = i;
                if (nx == -1) {
                    S.parent[r] = i;
                    break;
                }
                r = nx;
            }
        }
    rowk.clear();

    // column structures: struct(j) = A'(>j, j) U children's structs \ {j}
    std::vector<std::vector<int32_t>> st(n);
    std::vector<std::vector<int32_t>> children(n);
    for (int j = 0; j < n; j++)
        if (S.parent[j] >= 0) children[S.parent[j]].push_back(j);
    std::vector<int32_t> mark(n, -1);
    for (int j = 0; j < n; j++) {
        auto &s = st[j];
        mark[j] = j;
        for (int p = S.Ap[j]; p < S.Ap[j + 1]; p++) {
            int i = S.Ai[p];
            if (mark[i] != j) {
                mark[i] = j;
                s.push_back(i);
            }
        }
        for (int c : children[j]) {
            for (int i : st[c])
                if (mark[i] != j) {
                    mark[i] = j;
                    s.push_back(i);
                }
            // a child's structure is no longer needed once merged
            std::vector<int32_t>().swap(st[c]);
        }
        std::sort(s.begin(), s.end());
        // store into CSC now (children's lists are released as we go)
        if (j == 0) S.Lp.assign(1, 0);
        S.Lp.push_back(S.Lp.back() + (int32_t)s.size());
        S.Li.insert(S.Li.end(), s.begin(), s.end());
    }
    // CSR view of L's strict lower part
    S.Rp.assign(n + 1, 0);
    for (int64_t p = 0; p < S.nnzL(); p++) S.Rp[S.Li[p] + 1]++;
    for (int i = 0; i < n; i++) S.Rp[i + 1] += S.Rp[i];
    S.Rj.assign(S.nnzL(), 0);
    S.Rmap.assign(S.nnzL(), 0);
    {
        std::vector<int32_t> fill(S.Rp.begin(), S.Rp.end() - 1);
        for (int j = 0; j < n; j++)
            for (int p = S.Lp[j]; p < S.Lp[j + 1]; p++) {
                int i = S.Li[p];
                S.Rj[fill[i]] = j;
                S.Rmap[fill[i]] = p;
                fill[i]++;
            }
    }
    // dissection blocks, dense offsets, level schedule, external entry ranges
    S.bstart = nd.bstart;
    S.bheight = nd.bheight;
    S.bfirst = nd.bfirst;
    const int nb = (int)S.bheight.size();
    S.blk.assign(n, 0);
    S.doff.assign(nb + 1, 0);
    int nl = 0;
    for (int b = 0; b < nb; b++) {
        const int w = S.bstart[b + 1] - S.bstart[b];
        for (int r = S.bstart[b]; r < S.bstart[b + 1]; r++) S.blk[r] = b;
        S.doff[b + 1] = S.doff[b] + (int64_t)w * w;
        nl = std::max(nl, S.bheight[b] + 1);
    }
    S.ndense = S.doff[nb];
    S.lptr.assign(nl + 1, 0);
    for (int b = 0; b < nb; b++) S.lptr[S.bheight[b] + 1] += S.bstart[b + 1] - S.bstart[b];
    for (int l = 0; l < nl; l++) S.lptr[l + 1] += S.lptr[l];
    S.lrow.assign(n, 0);
    {
        std::vector<int32_t> fill(S.lptr.begin(), S.lptr.end() - 1);
        for (int b = 0; b < nb; b++)
            for (int r = S.bstart[b]; r < S.bstart[b + 1]; r++) S.lrow[fill[S.bheight[b]]++] = r;
    }
    S.fext.assign(n, 0);
    S.bext.assign(n, 0);
    for (int j = 0; j < n; j++) {
        const int b0 = S.bstart[S.blk[j]], b1 = S.bstart[S.blk[j] + 1];
        int e = S.Rp[j];
        while (e < S.Rp[j + 1] && S.Rj[e] < b0) e++;
        S.fext[j] = e;
        int p = S.Lp[j];
        while (p < S.Lp[j + 1] && S.Li[p] < b1) p++;
        S.bext[j] = p;
        // the level schedule needs every external entry to reference a block
        // of smaller height (a dissection descendant)
        for (int q = S.Rp[j]; q < e; q++)
            if (S.bheight[S.blk[S.Rj[q]]] >= S.bheight[S.blk[j]]) S.blocks_ok = false;
    }
    return S;
}

bool ldl_numeric(const LdlSymbolic &S, const std::vector<cd> &vals, std::vector<cd> &D,
                 std::vector<cd> &Lx) {
    const int n = S.n;
    D.assign(n, cd(0));
    Lx.assign(S.nnzL(), cd(0));
    std::vector<cd> w(n, cd(0));
    std::vector<int32_t> head(n, -1), link(n, -1), next(n, 0);
    for (int j = 0; j < n; j++) {
        for (int p = S.Ap[j]; p < S.Ap[j + 1]; p++) w[S.Ai[p]] = vals[S.Asrc[p]];
        // left-looking updates from columns k with L(j,k) != 0
        int k = head[j];
        head[j] = -1;
        while (k != -1) {
            int knext = link[k];
            int pos = next[k];
            cd f = Lx[pos] * D[k];
            for (int p = pos; p < S.Lp[k + 1]; p++) w[S.Li[p]] -= Lx[p] * f;
            next[k] = pos + 1;
            if (next[k] < S.Lp[k + 1]) {
                int r = S.Li[next[k]];
                link[k] = head[r];
                head[r] = k;
            }
            k = knext;
        }
        const cd dj = w[j];
        if (dj == cd(0) || !std::isfinite(dj.real()) || !std::isfinite(dj.imag())) return false;
        D[j] = dj;
        w[j] = cd(0);
        for (int p = S.Lp[j]; p < S.Lp[j + 1]; p++) {
            Lx[p] = w[S.Li[p]] / dj;
            w[S.Li[p]] = cd(0);
        }
        if (S.Lp[j] < S.Lp[j + 1]) {
            next[j] = S.Lp[j];
            int r = S.Li[S.Lp[j]];
            link[j] = head[r];
            head[r] = j;
        }
    }
    return true;
}

void ldl_block_inverses(const LdlSymbolic &S, const std::vector<cd> &Lx, std::vector<cd> &invL,
                        std::vector<cd> &invLT) {
    invL.assign(S.ndense, cd(0));
    invLT.assign(S.ndense, cd(0));
    const int nb = (int)S.bheight.size();
    std::vector<cd> Lb;
    for (int b = 0; b < nb; b++) {
        const int s0 = S.bstart[b], w = S.bstart[b + 1] - s0;
        Lb.assign((size_t)w * w, cd(0));
        for (int c = 0; c < w; c++) {
            Lb[(size_t)c * w + c] = 1.0;
            for (int p = S.Lp[s0 + c]; p < S.Lp[s0 + c + 1]; p++) {
                const int i = S.Li[p] - s0;
                if (i < w) Lb[(size_t)i * w + c] = Lx[p];
            }
        }
        cd *X = &invL[S.doff[b]];
        // X = Lb^{-1}: column by column, forward substitution
        for (int c = 0; c < w; c++) {
            X[(size_t)c * w + c] = 1.0;
            for (int i = c + 1; i < w; i++) {
                cd acc = 0.0;
                for (int t = c; t < i; t++) acc += Lb[(size_t)i * w + t] * X[(size_t)t * w + c];
                X[(size_t)i * w + c] = -acc;
            }
        }
        cd *XT = &invLT[S.doff[b]];
        for (int i = 0; i < w; i++)
            for (int c = 0; c < w; c++) XT[(size_t)c * w + i] = X[(size_t)i * w + c];
    }
}

void ldl_solve_blocks_host(const LdlSymbolic &S, const std::vector<cd> &D,
                           const std::vector<cd> &Lx, const std::vector<cd> &invL,
                           const std::vector<cd> &invLT, const std::vector<cd> &b,
                           std::vector<cd> &x) {
    const int n = S.n, nl = (int)S.lptr.size() - 1;
    std::vector<cd> y(n), z(n);
    for (int i = 0; i < n; i++) y[i] = b[S.perm[i]];
    for (int l = 0; l < nl; l++) {
        for (int r = S.lptr[l]; r < S.lptr[l + 1]; r++) {
            const int j = S.lrow[r];
            for (int e = S.Rp[j]; e < S.fext[j]; e++) y[j] -= Lx[S.Rmap[e]] * y[S.Rj[e]];
        }
        for (int r = S.lptr[l]; r < S.lptr[l + 1]; r++) {
            const int i = S.lrow[r], bb = S.blk[i], s0 = S.bstart[bb],
                      w = S.bstart[bb + 1] - s0;
            cd acc = 0.0;
            for (int t = 0; t <= i - s0; t++) acc += invL[S.doff[bb] + (i - s0) * w + t] * y[s0 + t];
            z[i] = acc;
        }
        for (int r = S.lptr[l]; r < S.lptr[l + 1]; r++) y[S.lrow[r]] = z[S.lrow[r]];
    }
    for (int i = 0; i < n; i++) y[i] /= D[i];
    for (int l = nl - 1; l >= 0; l--) {
        for (int r = S.lptr[l]; r < S.lptr[l + 1]; r++) {
            const int j = S.lrow[r];
            for (int p = S.bext[j]; p < S.Lp[j + 1]; p++) y[j] -= Lx[p] * y[S.Li[p]];
        }
        for (int r = S.lptr[l]; r < S.lptr[l + 1]; r++) {
            const int i = S.lrow[r], bb = S.blk[i], s0 = S.bstart[bb],
                      w = S.bstart[bb + 1] - s0;
            cd acc = 0.0;
            for (int t = i - s0; t < w; t++) acc += invLT[S.doff[bb] + (i - s0) * w + t] * y[s0 + t];
            z[i] = acc;
        }
        for (int r = S.lptr[l]; r < S.lptr[l + 1]; r++) y[S.lrow[r]] = z[S.lrow[r]];
    }
    x.assign(n, cd(0));
    for (int i = 0; i < n; i++) x[S.perm[i]] = y[i];
}

namespace {

// The plan at cut height H (ok = false if a limit is exceeded or the
// structure is not the one the kernels assume).
LdlSplit split_at(const LdlSymbolic &S, int H, int sub_max_rows, int top_max_rows,
                  int phase_max_rows) {
    LdlSplit P;
    const int n = S.n, nb = (int)S.bheight.size();
    P.H = H;
    P.hmax = 0;
    for (int b = 0; b < nb; b++) P.hmax = std::max(P.hmax, (int)S.bheight[b]);
    // roots of the bottom subtrees (scan from the top: subtrees are contiguous)
    std::vector<int32_t> roots, topb, sub_of(n, -1);
    for (int b = nb - 1; b >= 0;) {
        if (S.bheight[b] < H) {
            roots.push_back(b);
            b = S.bfirst[b] - 1;
        } else {
            topb.push_back(b);
            b--;
        }
    }
    std::reverse(roots.begin(), roots.end());
    std::reverse(topb.begin(), topb.end());
    P.nsub = (int)roots.size();
    for (int s = 0; s < P.nsub; s++) {
        const int root = roots[s], r0 = S.bstart[S.bfirst[root]], r1 = S.bstart[root + 1];
        if (r1 - r0 > sub_max_rows) return P;
        P.max_sub_rows = std::max(P.max_sub_rows, r1 - r0);
        P.sub_r0.push_back(r0);
        P.sub_r1.push_back(r1);
        for (int r = r0; r < r1; r++) sub_of[r] = s;
        std::vector<std::vector<int32_t>> byh(H);
        for (int b = S.bfirst[root]; b <= root; b++)
            for (int r = S.bstart[b]; r < S.bstart[b + 1]; r++) byh[S.bheight[b]].push_back(r);
        for (int h = 0; h < H; h++) {
            if ((int)byh[h].size() > phase_max_rows) return P;
            P.sub_hptr.push_back((int32_t)P.srow.size());
            P.srow.insert(P.srow.end(), byh[h].begin(), byh[h].end());
        }
    }
    P.sub_hptr.push_back((int32_t)P.srow.size());
    // top part
    std::vector<int32_t> tl(n, -1);
    for (int b : topb)
        for (int r = S.bstart[b]; r < S.bstart[b + 1]; r++) P.top_row.push_back(r);
    P.ntop = (int)P.top_row.size();
    if (P.ntop > top_max_rows) return P;
    for (int t = 0; t < P.ntop; t++) tl[P.top_row[t]] = t;
    if (P.ntop > 0) {
        std::vector<std::vector<int32_t>> byh(P.hmax - H + 1);
        for (int t = 0; t < P.ntop; t++) byh[S.bheight[S.blk[P.top_row[t]]] - H].push_back(t);
        for (auto &v : byh) {
            if ((int)v.size() > phase_max_rows) return P;
            P.top_hptr.push_back((int32_t)P.tlist.size());
            P.tlist.insert(P.tlist.end(), v.begin(), v.end());
        }
        P.top_hptr.push_back((int32_t)P.tlist.size());
    }
    // every row is in exactly one subtree or in the top
    for (int r = 0; r < n; r++)
        if ((sub_of[r] >= 0) == (tl[r] >= 0)) return P;
    // bottom rows: forward entries inside the own subtree, backward entries in
    // the own subtree first, then in the top part
    P.bsplit.assign(n, 0);
    for (int s = 0; s < P.nsub; s++)
        for (int j = P.sub_r0[s]; j < P.sub_r1[s]; j++) {
            for (int q = S.Rp[j]; q < S.fext[j]; q++)
                if (S.Rj[q] < P.sub_r0[s] || S.Rj[q] >= j) return P;
            int e = S.bext[j];
            while (e < S.Lp[j + 1] && S.Li[e] < P.sub_r1[s]) e++;
            for (int e2 = e; e2 < S.Lp[j + 1]; e2++)
                if (tl[S.Li[e2]] < 0) return P;
            P.bsplit[j] = e;
        }
    // top rows: forward entries by subtree (contiguous column ranges) and in the
    // top part; backward entries all in the top part
    P.part_b.assign((size_t)P.nsub * P.ntop, 0);
    P.part_e.assign((size_t)P.nsub * P.ntop, 0);
    P.tf_ptr.push_back(0);
    P.tb_ptr.push_back(0);
    for (int t = 0; t < P.ntop; t++) {
        const int j = P.top_row[t];
        int counted = 0;
        for (int s = 0; s < P.nsub; s++) {
            const int32_t *c0 = S.Rj.data() + S.Rp[j], *c1 = S.Rj.data() + S.fext[j];
            const int b = (int)(std::lower_bound(c0, c1, P.sub_r0[s]) - S.Rj.data());
            const int e = (int)(std::lower_bound(c0, c1, P.sub_r1[s]) - S.Rj.data());
            P.part_b[(size_t)s * P.ntop + t] = b;
            P.part_e[(size_t)s * P.ntop + t] = e;
            counted += e - b;
        }
        for (int q = S.Rp[j]; q < S.fext[j]; q++)
            if (tl[S.Rj[q]] >= 0) {
                P.tf_pos.push_back(q);
                P.tf_col.push_back(tl[S.Rj[q]]);
                counted++;
            }
        if (counted != S.fext[j] - S.Rp[j]) return P;
        P.tf_ptr.push_back((int32_t)P.tf_pos.size());
        for (int e = S.bext[j]; e < S.Lp[j + 1]; e++) {
            if (tl[S.Li[e]] < 0) return P;
            P.tb_pos.push_back(e);
            P.tb_row.push_back(tl[S.Li[e]]);
        }
        P.tb_ptr.push_back((int32_t)P.tb_pos.size());
    }
    P.ok = true;
    return P;
}

}   // namespace

LdlSplit ldl_split_plan(const LdlSymbolic &S, int sub_max_rows, int top_max_rows,
                        int phase_max_rows) {
    int hmax = 0;
    for (int h : S.bheight) hmax = std::max(hmax, h);
    // the largest cut height that fits: the smallest top part
    for (int H = hmax + 1; H >= 1; H--) {
        LdlSplit P = split_at(S, H, sub_max_rows, top_max_rows, phase_max_rows);
        if (P.ok) return P;
    }
    return LdlSplit{};
}

void ldl_solve_split_host(const LdlSymbolic &S, const LdlSplit &P, const std::vector<cd> &D,
                          const std::vector<cd> &Lx, const std::vector<cd> &invL,
                          const std::vector<cd> &invLT, const std::vector<cd> &b,
                          std::vector<cd> &x) {
    const int n = S.n;
    std::vector<cd> y(n), z(n), part((size_t)P.nsub * P.ntop);
    auto dense = [&](const int32_t *rows, int cnt, bool fwd) {
        for (int k = 0; k < cnt; k++) {
            const int i = rows[k], bb = S.blk[i], s0 = S.bstart[bb], w = S.bstart[bb + 1] - s0;
            cd acc = 0.0;
            if (fwd)
                for (int t = 0; t <= i - s0; t++) acc += invL[S.doff[bb] + (i - s0) * w + t] * y[s0 + t];
            else
                for (int t = i - s0; t < w; t++) acc += invLT[S.doff[bb] + (i - s0) * w + t] * y[s0 + t];
            z[i] = acc;
        }
        for (int k = 0; k < cnt; k++) y[rows[k]] = z[rows[k]];
    };
    // bottom, forward, and the partial sums of the top rows
    for (int s = 0; s < P.nsub; s++) {
        for (int h = 0; h < P.H; h++) {
            const int a = P.sub_hptr[s * P.H + h], e = P.sub_hptr[s * P.H + h + 1];
            for (int k = a; k < e; k++) {
                const int j = P.srow[k];
                cd acc = 0.0;
                for (int q = S.Rp[j]; q < S.fext[j]; q++) acc += Lx[S.Rmap[q]] * y[S.Rj[q]];
                y[j] = b[S.perm[j]] - acc;
            }
            dense(P.srow.data() + a, e - a, true);
        }
        for (int t = 0; t < P.ntop; t++) {
            cd acc = 0.0;
            for (int q = P.part_b[(size_t)s * P.ntop + t]; q < P.part_e[(size_t)s * P.ntop + t]; q++)
                acc += Lx[S.Rmap[q]] * y[S.Rj[q]];
            part[(size_t)s * P.ntop + t] = acc;
        }
    }
    // top, forward then backward
    const int nht = (int)P.top_hptr.size() - 1;
    std::vector<int32_t> rows;
    for (int h = 0; h < nht; h++) {
        rows.clear();
        for (int k = P.top_hptr[h]; k < P.top_hptr[h + 1]; k++) {
            const int t = P.tlist[k], j = P.top_row[t];
            cd acc = 0.0;
            for (int s = 0; s < P.nsub; s++) acc += part[(size_t)s * P.ntop + t];
            for (int q = P.tf_ptr[t]; q < P.tf_ptr[t + 1]; q++)
                acc += Lx[S.Rmap[P.tf_pos[q]]] * y[P.top_row[P.tf_col[q]]];
            y[j] = b[S.perm[j]] - acc;
            rows.push_back(j);
        }
        dense(rows.data(), (int)rows.size(), true);
    }
    for (int h = nht - 1; h >= 0; h--) {
        rows.clear();
        for (int k = P.top_hptr[h]; k < P.top_hptr[h + 1]; k++) {
            const int t = P.tlist[k], j = P.top_row[t];
            cd acc = 0.0;
            for (int q = P.tb_ptr[t]; q < P.tb_ptr[t + 1]; q++)
                acc += Lx[P.tb_pos[q]] * y[P.top_row[P.tb_row[q]]];
            y[j] = y[j] / D[j] - acc;
            rows.push_back(j);
        }
        dense(rows.data(), (int)rows.size(), false);
    }
    // bottom, backward
    for (int s = 0; s < P.nsub; s++)
        for (int h = P.H - 1; h >= 0; h--) {
            const int a = P.sub_hptr[s * P.H + h], e = P.sub_hptr[s * P.H + h + 1];
            for (int k = a; k < e; k++) {
                const int j = P.srow[k];
                cd acc = 0.0;
                for (int q = S.bext[j]; q < S.Lp[j + 1]; q++) acc += Lx[q] * y[S.Li[q]];
                y[j] = y[j] / D[j] - acc;
            }
            dense(P.srow.data() + a, e - a, false);
        }
    x.assign(n, cd(0));
    for (int i = 0; i < n; i++) x[S.perm[i]] = y[i];
}

void ldl_solve_host(const LdlSymbolic &S, const std::vector<cd> &D, const std::vector<cd> &Lx,
                    const std::vector<cd> &b, std::vector<cd> &x) {
    const int n = S.n;
    std::vector<cd> y(n);
    for (int i = 0; i < n; i++) y[i] = b[S.perm[i]];
    for (int j = 0; j < n; j++)
        for (int p = S.Lp[j]; p < S.Lp[j + 1]; p++) y[S.Li[p]] -= Lx[p] * y[j];
    for (int i = 0; i < n; i++) y[i] /= D[i];
    for (int j = n - 1; j >= 0; j--)
        for (int p = S.Lp[j]; p < S.Lp[j + 1]; p++) y[j] -= Lx[p] * y[S.Li[p]];
    x.assign(n, cd(0));
    for (int i = 0; i < n; i++) x[S.perm[i]] = y[i];
}

}   // namespace bem

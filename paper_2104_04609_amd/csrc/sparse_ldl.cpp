// Sparse complex-symmetric LDL^T: nested dissection, symbolic analysis,
// left-looking numeric factorisation, level schedules for the GPU solves.
#include "sparse_ldl.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace bem {

namespace {

void dissect(std::vector<int32_t> &vs, const std::vector<int32_t> &ptr,
             const std::vector<int32_t> &col, const std::vector<double> &xyz,
             std::vector<int32_t> &side, std::vector<int32_t> &order, int leaf) {
    if ((int)vs.size() <= leaf) {
        order.insert(order.end(), vs.begin(), vs.end());
        return;
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
        order.insert(order.end(), vs.begin(), vs.end());
        return;
    }
    std::sort(A.begin(), A.end());
    std::sort(B.begin(), B.end());
    std::sort(S.begin(), S.end());
    dissect(A, ptr, col, xyz, side, order, leaf);
    dissect(B, ptr, col, xyz, side, order, leaf);
    order.insert(order.end(), S.begin(), S.end());
}

}   // namespace

std::vector<int32_t> nested_dissection(int n, const std::vector<int32_t> &ptr,
                                       const std::vector<int32_t> &col,
                                       const std::vector<double> &xyz,
                                       const std::vector<int32_t> &group, int leaf) {
    std::vector<int32_t> order, side(n, 0);
    order.reserve(n);
    int ng = 0;
    for (int v = 0; v < n; v++) ng = std::max(ng, group[v] + 1);
    for (int g = 0; g < ng; g++) {
        std::vector<int32_t> vs;
        for (int v = 0; v < n; v++)
            if (group[v] == g) vs.push_back(v);
        dissect(vs, ptr, col, xyz, side, order, leaf);
    }
    return order;
}

LdlSymbolic ldl_symbolic(int n, const std::vector<int32_t> &ptr,
                         const std::vector<int32_t> &col, const std::vector<int32_t> &perm) {
    LdlSymbolic S;
    S.n = n;
    S.perm = perm;
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
    // level schedules
    std::vector<int32_t> h(n, 0), d(n, 0);
    for (int j = 0; j < n; j++)
        if (S.parent[j] >= 0) h[S.parent[j]] = std::max(h[S.parent[j]], h[j] + 1);
    for (int j = n - 1; j >= 0; j--) d[j] = S.parent[j] >= 0 ? d[S.parent[j]] + 1 : 0;
    auto schedule = [n](const std::vector<int32_t> &lev, std::vector<int32_t> &lp,
                        std::vector<int32_t> &rows) {
        int nl = 0;
        for (int j = 0; j < n; j++) nl = std::max(nl, lev[j] + 1);
        lp.assign(nl + 1, 0);
        for (int j = 0; j < n; j++) lp[lev[j] + 1]++;
        for (int l = 0; l < nl; l++) lp[l + 1] += lp[l];
        rows.assign(n, 0);
        std::vector<int32_t> fill(lp.begin(), lp.end() - 1);
        for (int j = 0; j < n; j++) rows[fill[lev[j]]++] = j;
    };
    schedule(h, S.fptr, S.frow);
    schedule(d, S.bptr, S.brow);
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

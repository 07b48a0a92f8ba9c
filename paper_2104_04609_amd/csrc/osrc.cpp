// OSRC preconditioner (Sec. 2.6, Sec. 2.7 of the paper): host set-up of the
// shifted sparse factorisations and the stream-ordered application.
//
//   L_DtN = ik (I + X)^{1/2},  L_NtD = (1/ik) (I + X)^{-1/2},  X = Delta_Gamma / k_eps^2
//
// with the square root replaced by the N_p-term Pade approximant with
// branch-cut rotation theta,  sqrt(1+z) ~ C_0 + sum_j A_j z / (1 + B_j z).
// In P1 Galerkin form (mass M, stiffness S, X_h = -M^{-1} S / k_eps^2):
//   R(X_h) u = M^{-1} [C_0 M u - (1/k_eps^2) S sum_j A_j (M - (B_j/k_eps^2) S)^{-1} M u]
//   L_DtN u = ik R(X_h) u,   L_NtD u = (1/ik) R(X_h) (M - S/k_eps^2)^{-1} M u.
// The Pade coefficients follow the rotated approximant of Milinazzo, Zala and
// Brooke with the Antoine-Darbas rotation (the paper cites it without the
// formulas):  a_j = 2/(2N_p+1) sin^2(j pi/(2N_p+1)), b_j = cos^2(j pi/(2N_p+1)),
//   C_0 = e^{i theta/2} [1 + sum_j a_j (e^{-i theta} - 1)/(1 + b_j (e^{-i theta} - 1))],
//   A_j = e^{-i theta/2} a_j / (1 + b_j (e^{-i theta} - 1))^2,
//   B_j = e^{-i theta} b_j / (1 + b_j (e^{-i theta} - 1)).
// Applied in partial-fraction form: with
// M^{-1} S (M - beta S)^{-1} = [(M - beta S)^{-1} - M^{-1}] / beta,
//   R(X_h) u = C_0' u - sum_j (A_j / B_j) (M - (B_j/k_eps^2) S)^{-1} M u,
//   C_0' = C_0 + sum_j A_j / B_j,
// and, with (I + B X)^{-1} (I + X)^{-1} = [(I + X)^{-1} - B (I + B X)^{-1}] / (1 - B)
// (B_j != 1 since b_j < 1), the NtD operator over the same shifts,
//   R(X_h) (I + X_h)^{-1} = [C_0 - sum_j A_j/(1 - B_j)] (I + X_h)^{-1}
//                           + sum_j A_j/(1 - B_j) (I + B_j X_h)^{-1},
// (I + B X_h)^{-1} u = (M - (B/k_eps^2) S)^{-1} M u.  So one application is
// one batch of 2 N_p + 2 solves on the two weak inputs (two stages above 16
// Pade terms, where the task list is full) and no stiffness products.
// All N_p + 2 systems (N_p shifts, M - S/k_eps^2, M) share the vertex-graph
// pattern, one ordering and one symbolic factorisation; each is factorised
// once (complex-symmetric LDL^T) and kept on the device (Sec. 2.7: a sparse
// factorisation computed once and reused every iteration).
#include <cmath>
#include <complex>
#include <algorithm>
#include <thread>

#include "osrc_internal.h"

namespace bem {

void OsrcDeleter::operator()(OsrcState *p) const { delete p; }
void OsrcSymDeleter::operator()(OsrcSymbolicState *p) const { delete p; }

int64_t SplitSchedule::bytes() const {
    return sub_r0.bytes() + sub_r1.bytes() + sub_hptr.bytes() + srow.bytes() + top_row.bytes() +
           top_hptr.bytes() + tlist.bytes() + part_b.bytes() + part_e.bytes() + tf_ptr.bytes() +
           tf_pos.bytes() + tf_col.bytes() + tb_ptr.bytes() + tb_pos.bytes() + tb_row.bytes() +
           bsplit.bytes() + sdesc.bytes();
}
int64_t OsrcSymbolicState::bytes() const {
    return gptr_d.bytes() + gcol_d.bytes() + perm_d.bytes() + Rj_d.bytes() + Li_d.bytes() +
           Mv_d.bytes() + Sv_d.bytes() + jrow_d.bytes() + lrowd_d.bytes() + lblkd_d.bytes() + split.bytes() +
           bottom[0].bytes() + bottom[1].bytes() + bottom[2].bytes() + bottom[3].bytes();
}
int64_t OsrcState::bytes() const {
    return cvert.bytes() + ikv.bytes() + iikv.bytes() + Dinv.bytes() + Lcsr.bytes() +
           Lcsc.bytes() + invL.bytes() + invLT.bytes() + work.bytes() + obuf.bytes() +
           wbuf.bytes();
}

// Both operators' solves in one batch (2 N_p + 2 systems) when the task
// list holds them, else two stages (N_p + 2, then N_p systems).
bool osrc_one_stage(int np) { return 2 * np + 2 <= PADE_MAX + 2; }
int osrc_tasks(int np) { return osrc_one_stage(np) ? 2 * np + 2 : np + 2; }
// solve outputs per right-hand side: one stage s_0..s_{np-1}, u, s'_0..
// s'_{np-1}, v; two stages s_0..s_{np-1}, u, v, M v
int64_t osrc_obuf_len(int np, int64_t n) { return (osrc_one_stage(np) ? 2 * np + 2 : np + 3) * n; }

void OsrcState::ensure_batch(int R) {
    if (R <= batch) return;
    const size_t n = cvert.n;
    work.alloc((size_t)R * osrc_tasks(np) * wlen);
    obuf.alloc((size_t)R * osrc_obuf_len(np, n));
    wbuf.alloc((size_t)R * 2 * n);
    batch = R;
}
int64_t osrc_bytes(const OsrcState &st) { return st.bytes(); }

OsrcStats osrc_stats(const bem_mesh *m, const OsrcState &st) {
    const OsrcSymbolicState &sy = *m->osrc_sym;
    const LdlSymbolic &S = sy.sym;
    OsrcStats o;
    o.n = sy.n;
    o.np = st.np;
    o.nfactors = st.nfactors;
    o.solves = 2 * st.np + 2;
    o.nnz_l = S.nnzL();
    o.nnz_ext = 0;
    for (int j = 0; j < sy.n; j++) o.nnz_ext += (S.fext[j] - S.Rp[j]) + (S.Lp[j + 1] - S.bext[j]);
    o.nnz_ext /= 2;   // forward and backward sweeps visit the same entries
    o.ndense = S.ndense;
    o.mass_nnz = (int64_t)sy.gcol.size();
    o.factor_bytes = st.Dinv.bytes() + st.Lcsr.bytes() + st.Lcsc.bytes() + st.invL.bytes() +
                     st.invLT.bytes();
    // one single-vector apply: per block solve the off-block entries of L (rows)
    // and L^T (columns) with their indices, both dense inverses, D^{-1}, the
    // input and the output; two mass products (three with two stages; 8-byte
    // values, column indices, row pointers, input, output); two Pade sums
    // (np + 1 inputs, one output)
    const int64_t c16 = 16, n = o.n;
    const int64_t per_solve = 2 * o.nnz_ext * (c16 + 4) + 2 * o.ndense * c16 + n * c16 + 2 * n * c16;
    const int64_t spmv = o.mass_nnz * 12 + (n + 1) * 4 + 2 * n * c16;
    const int64_t sums = (int64_t)(st.np + 2) * n * c16;
    o.bytes_per_apply = o.solves * per_solve + (osrc_one_stage(st.np) ? 2 : 3) * spmv + 2 * sums;
    return o;
}
int64_t osrc_sym_bytes(const OsrcSymbolicState &st) { return st.bytes(); }

namespace {

using cdd = std::complex<double>;

double2 d2(cdd z) { return make_double2(z.real(), z.imag()); }

OsrcSymbolicState &symbolic(bem_mesh *m) {
    if (m->osrc_sym) return *m->osrc_sym;
    auto st = std::unique_ptr<OsrcSymbolicState, OsrcSymDeleter>(new OsrcSymbolicState());
    const int n = (int)m->N;
    st->n = n;
    // P1 vertex graph (vertices sharing a triangle), sorted, incl. diagonal
    std::vector<std::vector<int32_t>> adj(n);
    for (int64_t t = 0; t < m->T; t++)
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) adj[m->tri[3 * t + a]].push_back(m->tri[3 * t + b]);
    st->gptr.assign(n + 1, 0);
    for (int i = 0; i < n; i++) {
        auto &r = adj[i];
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        st->gptr[i + 1] = st->gptr[i] + (int32_t)r.size();
    }
    st->gcol.reserve(st->gptr[n]);
    for (int i = 0; i < n; i++) st->gcol.insert(st->gcol.end(), adj[i].begin(), adj[i].end());
    // mass M_ab = |tau|/12 (1 + delta_ab); stiffness S_ab = |tau| grad phi_a . grad phi_b
    // (curl phi = n x grad phi preserves the dot product)
    st->Mv.assign(st->gptr[n], 0.0);
    st->Sv.assign(st->gptr[n], 0.0);
    auto pos = [&](int i, int j) {
        auto b = st->gcol.begin() + st->gptr[i], e = st->gcol.begin() + st->gptr[i + 1];
        return (int)(std::lower_bound(b, e, j) - st->gcol.begin());
    };
    for (int64_t t = 0; t < m->T; t++) {
        const double ar = m->area[t];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                int e = pos(m->tri[3 * t + a], m->tri[3 * t + b]);
                st->Mv[e] += ar / 12.0 * (a == b ? 2.0 : 1.0);
                const double *ca = &m->curl[9 * t + 3 * a], *cb = &m->curl[9 * t + 3 * b];
                st->Sv[e] += ar * (ca[0] * cb[0] + ca[1] * cb[1] + ca[2] * cb[2]);
            }
    }
    const NdOrder nd = nested_dissection(n, st->gptr, st->gcol, m->P, m->vobj);
    st->sym = ldl_symbolic(n, st->gptr, st->gcol, nd);
    const LdlSymbolic &S = st->sym;
    if (!S.blocks_ok) fail(BEM_E_UNSUPPORTED, "dissection blocks violate the level order");
    st->gptr_d.upload(st->gptr);
    st->gcol_d.upload(st->gcol);
    st->Mv_d.upload(st->Mv);
    st->Sv_d.upload(st->Sv);
    st->perm_d.upload(S.perm);
    st->Rj_d.upload(S.Rj);
    st->Li_d.upload(S.Li);
    // blocks per level, external entry ranges, dense offsets
    const int nb = (int)S.bheight.size(), nl = (int)S.lptr.size() - 1;
    for (int b = 0; b < nb; b++)
        if (S.bstart[b + 1] - S.bstart[b] > LDL_MAX_BLOCK)
            fail(BEM_E_UNSUPPORTED, "dissection block larger than the solve workgroup can hold");
    std::vector<int32_t> lbptr(nl + 1, 0), lblk(nb);
    for (int b = 0; b < nb; b++) lbptr[S.bheight[b] + 1]++;
    for (int l = 0; l < nl; l++) lbptr[l + 1] += lbptr[l];
    {
        std::vector<int32_t> fill(lbptr.begin(), lbptr.end() - 1);
        for (int b = 0; b < nb; b++) lblk[fill[S.bheight[b]]++] = b;
    }
    st->lbcount.assign(nl, 0);
    st->lrcount.assign(nl, 0);
    for (int l = 0; l < nl; l++) {
        st->lbcount[l] = lbptr[l + 1] - lbptr[l];
        st->lrcount[l] = S.lptr[l + 1] - S.lptr[l];
    }
    // row and block descriptors (one load per row / block in the solve kernels)
    if (S.ndense >= ((int64_t)1 << 31)) fail(BEM_E_UNSUPPORTED, "dense block inverses too large");
    std::vector<LdlRow> jrow(n);
    for (int j = 0; j < n; j++) {
        const int b = S.blk[j], s0 = S.bstart[b];
        jrow[j] = LdlRow{j, S.perm[j], s0, S.bstart[b + 1] - s0, S.Rp[j], S.fext[j], S.bext[j],
                         S.Lp[j + 1], (int)S.doff[b], j - s0, 0, 0};
    }
    std::vector<LdlRow> lrowd(S.lrow.size());
    for (size_t r = 0; r < S.lrow.size(); r++) lrowd[r] = jrow[S.lrow[r]];
    std::vector<int4> lblkd(nb);
    for (int i = 0; i < nb; i++) {
        const int b = lblk[i];
        lblkd[i] = make_int4(S.bstart[b], S.bstart[b + 1] - S.bstart[b], (int)S.doff[b], 0);
    }
    st->jrow_d.upload(jrow);
    st->lrowd_d.upload(lrowd);
    st->lblkd_d.upload(lblkd);
    st->lptr_h = S.lptr;
    st->lbptr_h = lbptr;
    st->lext_f.assign(nl, 0);
    st->lext_b.assign(nl, 0);
    for (int l = 0; l < nl; l++)
        for (int r = S.lptr[l]; r < S.lptr[l + 1]; r++) {
            const int j = S.lrow[r];
            st->lext_f[l] += S.fext[j] - S.Rp[j];
            st->lext_b[l] += S.Lp[j + 1] - S.bext[j];
        }
    // two-part schedules: bottom subtrees in LDS, the top part by the level
    // kernels (or, in the form with partial sums, in one workgroup when its
    // own work is small, else level by level)
    st->wlen = 2 * (int64_t)n;   // y, z
    const Tuning &tn = tuning();
    auto make_split = [&](SplitSchedule &sc, int sub_rows, bool top_levels) {
        // rows of one height are staged in LDS next to the subtree's rows
        const int phase =
            std::min(4096, (int)((ldl_split_max_lds() - 16 * (int64_t)sub_rows - 32) / 20));
        if (phase < 64) return;
        LdlSplit P = ldl_split_plan(S, sub_rows, 8192, phase);
        if (!P.ok || P.H > LDL_SPLIT_MAX_H) return;
        int hrows = 0;
        for (int q = 0; q < P.nsub * P.H; q++)
            hrows = std::max(hrows, P.sub_hptr[q + 1] - P.sub_hptr[q]);
        for (size_t q = 0; q + 1 < P.top_hptr.size(); q++)
            hrows = std::max(hrows, P.top_hptr[q + 1] - P.top_hptr[q]);
        sc.hrows = hrows;
        sc.desc_lds = ldl_split_lds(P.max_sub_rows, hrows, P.max_sub_rows) <=
                              (size_t)ldl_split_max_lds()
                          ? 1
                          : 0;
        sc.top_levels = top_levels ? 1 : 0;
        sc.sub_r0.upload(P.sub_r0);
        sc.sub_r1.upload(P.sub_r1);
        sc.sub_hptr.upload(P.sub_hptr);
        sc.srow.upload(P.srow);
        sc.bsplit.upload(P.bsplit);
        if (!top_levels) {   // the top part's own tables and the partial sums
            sc.top_row.upload(P.top_row);
            sc.top_hptr.upload(P.top_hptr);
            sc.tlist.upload(P.tlist);
            sc.part_b.upload(P.part_b);
            sc.part_e.upload(P.part_e);
            sc.tf_ptr.upload(P.tf_ptr);
            sc.tf_pos.upload(P.tf_pos);
            sc.tf_col.upload(P.tf_col);
            sc.tb_ptr.upload(P.tb_ptr);
            sc.tb_pos.upload(P.tb_pos);
            sc.tb_row.upload(P.tb_row);
        }
        std::vector<LdlRow> sd(P.srow.size());
        for (size_t k = 0; k < P.srow.size(); k++) {
            sd[k] = jrow[P.srow[k]];
            sd[k].bsplit = P.bsplit[P.srow[k]];
        }
        sc.sdesc.upload(sd);
        sc.plan = std::move(P);
    };
    // 1 (automatic; measured on the 10 242- and 40 962-vertex meshes): the
    // bottom-subtree schedule with the top levels one launch per level; plans
    // with subtrees of up to 512 .. 4096 rows, each batch taking the one of
    // up to OSRC_SUB_ROWS rows, or a larger one when that still gives
    // OSRC_SUB_MIN_GROUPS workgroups.
    // 2: the two-part solve with partial sums; 3: one bottom-subtree plan of
    // up to osrc.bottom_rows rows
    const int split_mode = tn.osrc_split.load();
    st->split_mode = split_mode;
    if (split_mode == 2) {
        int sub_rows = std::min(ldl_split_max_sub_rows(), 4096);
        if (tn.osrc_sub_rows.load() > 0)
            sub_rows = std::min(ldl_split_max_sub_rows(), tn.osrc_sub_rows.load());
        make_split(st->split, sub_rows, false);
        const LdlSplit &P = st->split.plan;
        if (P.ok) {
            int64_t top_dense = 0;
            for (int b = 0; b < nb; b++)
                if (S.bheight[b] >= P.H) {
                    const int64_t w = S.bstart[b + 1] - S.bstart[b];
                    top_dense += w * w;
                }
            const int64_t top_work = (int64_t)P.tf_pos.size() + (int64_t)P.tb_pos.size() + top_dense;
            st->split.top_single = ldl_split_lds(P.ntop, st->split.hrows, 0) <=
                                               (size_t)ldl_split_max_lds() &&
                                           top_work <= tn.osrc_top_single_work.load()
                                       ? 1
                                       : 0;
            st->wlen = 2 * (int64_t)n + (int64_t)P.nsub * P.ntop;
        }
    } else if (split_mode == 1) {
        for (int rows = 512; rows <= 4096; rows *= 2) {
            if (rows > ldl_split_max_sub_rows()) break;
            SplitSchedule &sc = st->bottom[st->nbottom];
            make_split(sc, rows, true);
            if (!sc.plan.ok) continue;
            sc.rows = rows;
            // keep only plans that differ from the previous one
            if (st->nbottom > 0 && st->bottom[st->nbottom - 1].plan.H == sc.plan.H) {
                sc = SplitSchedule();
                continue;
            }
            st->nbottom++;
        }
    } else if (split_mode == 3) {
        const int rows = tn.osrc_bottom_rows.load();
        make_split(st->bottom[0], std::min(ldl_split_max_sub_rows(), rows), true);
        if (st->bottom[0].plan.ok) st->nbottom = 1;
    }
    m->osrc_sym = std::move(st);
    return *m->osrc_sym;
}

// Schedule of one batched block solve of `ntasks` systems and nrhs vectors:
// a bottom-subtree plan, the two-part solve with partial sums or, with
// ok = 0, one launch per level.
LdlSplitDev split_view(const OsrcSymbolicState &sy, int ntasks, int nrhs) {
    LdlSplitDev P{};
    const SplitSchedule *sc = nullptr;
    if (sy.split_mode == 2 && sy.split.plan.ok) {
        sc = &sy.split;
    } else if (sy.nbottom > 0) {
        // subtrees of up to OSRC_SUB_ROWS rows, larger ones while they still
        // give OSRC_SUB_MIN_GROUPS workgroups
        sc = &sy.bottom[0];
        for (int i = 0; i < sy.nbottom; i++)
            if (sy.bottom[i].rows <= OSRC_SUB_ROWS) sc = &sy.bottom[i];
        for (int i = sy.nbottom - 1; i >= 0 && sy.bottom[i].rows > sc->rows; i--)
            if ((int64_t)sy.bottom[i].plan.nsub * ntasks * nrhs >= OSRC_SUB_MIN_GROUPS) {
                sc = &sy.bottom[i];
                break;
            }
    }
    if (!sc) return P;
    const LdlSplit &q = sc->plan;
    P.ok = 1;
    P.top_levels = sc->top_levels;
    P.H = q.H;
    P.nsub = q.nsub;
    P.ntop = q.ntop;
    P.nht = q.ntop > 0 ? (int)q.top_hptr.size() - 1 : 0;
    P.top_single = sc->top_single;
    P.sub_rows = q.max_sub_rows;
    P.hrows = sc->hrows;
    P.desc_lds = sc->desc_lds;
    P.sub_r0 = sc->sub_r0.p;
    P.sub_r1 = sc->sub_r1.p;
    P.sub_hptr = sc->sub_hptr.p;
    P.srow = sc->srow.p;
    P.sdesc = sc->sdesc.p;
    P.top_row = sc->top_row.p;
    P.top_hptr = sc->top_hptr.p;
    P.tlist = sc->tlist.p;
    P.part_b = sc->part_b.p;
    P.part_e = sc->part_e.p;
    P.tf_ptr = sc->tf_ptr.p;
    P.tf_pos = sc->tf_pos.p;
    P.tf_col = sc->tf_col.p;
    P.tb_ptr = sc->tb_ptr.p;
    P.tb_pos = sc->tb_pos.p;
    P.tb_row = sc->tb_row.p;
    P.bsplit = sc->bsplit.p;
    return P;
}

LdlDev ldl_view(const OsrcSymbolicState &sy, const OsrcState &st) {
    LdlDev L;
    L.n = sy.n;
    L.nnz = sy.sym.nnzL();
    L.ndense = sy.sym.ndense;
    L.perm = sy.perm_d.p;
    L.Rj = sy.Rj_d.p;
    L.Li = sy.Li_d.p;
    L.nlev = (int)sy.lbcount.size();
    L.lbcount = sy.lbcount.data();
    L.lrcount = sy.lrcount.data();
    L.Dinv = st.Dinv.p;
    L.Lcsr = st.Lcsr.p;
    L.Lcsc = st.Lcsc.p;
    L.invL = st.invL.p;
    L.invLT = st.invLT.p;
    L.wlen = sy.wlen;
    L.jrow = sy.jrow_d.p;
    L.lrowd = sy.lrowd_d.p;
    L.lblkd = sy.lblkd_d.p;
    L.lptr_h = sy.lptr_h.data();
    L.lbptr_h = sy.lbptr_h.data();
    L.lext_f = sy.lext_f.data();
    L.lext_b = sy.lext_b.data();
    return L;
}

}   // namespace

void osrc_prepare(bem_mesh *m) { (void)symbolic(m); }

int64_t osrc_state_bytes(bem_mesh *m, int np, int R) {
    const OsrcSymbolicState &sy = symbolic(m);
    const int64_t n = sy.n, nnz = sy.sym.nnzL(), nd = sy.sym.ndense, nf = np + 2;
    // cvert, Dinv, L (CSR + CSC), dense block inverses (+ transposes); per
    // right-hand side work, outputs and weak vectors; complex128 each
    return (int64_t)sizeof(double2) *
           (n + nf * (n + 2 * nnz + 2 * nd) +
            (int64_t)R * (osrc_tasks(np) * sy.wlen + osrc_obuf_len(np, n) + 2 * n));
}

// Cache key of a state; k_obj with equal entries collapses to k (set to
// nullptr, k replaced by the common value).
static OsrcKey osrc_key(int np, double theta, double2 &k, const std::vector<double2> &keps_obj,
                 const std::vector<double2> *&k_obj) {
    OsrcKey key{np, theta, k.x, k.y, {}, {}};
    for (const double2 &ke : keps_obj) {
        key.keps.push_back(ke.x);
        key.keps.push_back(ke.y);
    }
    if (k_obj) {
        bool same = true;
        for (const double2 &ko : *k_obj) same = same && ko.x == (*k_obj)[0].x && ko.y == (*k_obj)[0].y;
        if (same) {
            k = (*k_obj)[0];
            key.kr = k.x;
            key.ki = k.y;
            k_obj = nullptr;
        } else {
            for (const double2 &ko : *k_obj) {
                key.kobj.push_back(ko.x);
                key.kobj.push_back(ko.y);
            }
        }
    }
    return key;
}

OsrcState *osrc_find(bem_mesh *m, int np, double theta, double2 k,
                     const std::vector<double2> &keps_obj) {
    if ((int)keps_obj.size() != m->nobj) fail(BEM_E_INVAL, "one k_eps per object expected");
    const std::vector<double2> *k_obj = nullptr;
    auto it = m->osrc_cache.find(osrc_key(np, theta, k, keps_obj, k_obj));
    return it == m->osrc_cache.end() ? nullptr : it->second.get();
}

int64_t osrc_work_len(const bem_mesh *m) { return m->osrc_sym->wlen; }

int64_t osrc_scratch_per_rhs(const bem_mesh *m, int np) {
    const int64_t n = m->osrc_sym->n, wlen = m->osrc_sym->wlen;
    return osrc_tasks(np) * wlen + osrc_obuf_len(np, n) + 2 * n;
}

OsrcScratch osrc_scratch_at(const bem_mesh *m, int np, int batch, double2 *base) {
    const int64_t n = m->osrc_sym->n, wlen = m->osrc_sym->wlen;
    double2 *obuf = base + (int64_t)batch * osrc_tasks(np) * wlen;
    return OsrcScratch{base, obuf, obuf + (int64_t)batch * osrc_obuf_len(np, n)};
}

OsrcState &osrc_get(bem_mesh *m, int np, double theta, double2 k,
                    const std::vector<double2> &keps_obj, hipStream_t s,
                    const std::vector<double2> *k_obj) {
    if ((int)keps_obj.size() != m->nobj) fail(BEM_E_INVAL, "one k_eps per object expected");
    if (k_obj && (int)k_obj->size() != m->nobj) fail(BEM_E_INVAL, "one k per object expected");
    const OsrcKey key = osrc_key(np, theta, k, keps_obj, k_obj);
    auto it = m->osrc_cache.find(key);
    if (it != m->osrc_cache.end()) return *it->second;
    OsrcSymbolicState &sy = symbolic(m);
    const int n = sy.n;
    auto st = std::unique_ptr<OsrcState, OsrcDeleter>(new OsrcState());
    st->np = np;
    st->wlen = sy.wlen;
    st->k = k;
    // Pade coefficients
    const cdd e = std::exp(cdd(0, -theta));
    cdd C0 = 0.0;
    std::vector<cdd> A(np), B(np);
    for (int j = 1; j <= np; j++) {
        const double sj = std::sin(j * M_PI / (2 * np + 1)), cj = std::cos(j * M_PI / (2 * np + 1));
        const double aj = 2.0 / (2 * np + 1) * sj * sj, bj = cj * cj;
        const cdd den = 1.0 + bj * (e - 1.0);
        C0 += aj * (e - 1.0) / den;
        A[j - 1] = std::exp(cdd(0, -theta / 2)) * aj / (den * den);
        B[j - 1] = e * bj / den;
    }
    C0 = std::exp(cdd(0, theta / 2)) * (1.0 + C0);
    st->pc.np = np;
    st->pc.C0 = d2(C0);
    for (int j = 0; j < np; j++) st->pc.A[j] = d2(A[j]);
    // partial-fraction coefficients: C_0' = C_0 + sum A_j/B_j, c_j = A_j/B_j
    cdd C0p = C0;
    st->pf.np = np;
    for (int j = 0; j < np; j++) {
        C0p += A[j] / B[j];
        st->pf.A[j] = d2(A[j] / B[j]);
    }
    st->pf.C0 = d2(C0p);
    // R(X)(I + X)^{-1} in partial fractions over (I + X)^{-1} and the same
    // shifts (B_j != 1 for b_j < 1):  [C_0 - sum_j A_j/(1 - B_j)] (I + X)^{-1}
    // + sum_j A_j/(1 - B_j) (I + B_j X)^{-1}; kept as C_0 - sum_j A_j s_j with
    // the signs of the Pade sum kernel
    cdd D0 = C0;
    st->qf.np = np;
    for (int j = 0; j < np; j++) {
        const cdd E = A[j] / (1.0 - B[j]);
        D0 -= E;
        st->qf.A[j] = d2(-E);
    }
    st->qf.C0 = d2(D0);
    st->B.resize(np);
    for (int j = 0; j < np; j++) st->B[j] = d2(B[j]);
    // 1/k_eps^2 per vertex (object)
    std::vector<double2> cv(n);
    std::vector<cdd> cobj(m->nobj);
    for (int o = 0; o < m->nobj; o++) {
        const cdd ke(keps_obj[o].x, keps_obj[o].y);
        cobj[o] = 1.0 / (ke * ke);
    }
    for (int v = 0; v < n; v++) cv[v] = d2(cobj[m->vobj[v]]);
    st->cvert.upload(cv);
    if (k_obj) {   // ik and 1/(ik) of each vertex's object
        std::vector<double2> a(n), ai(n);
        for (int v = 0; v < n; v++) {
            const cdd ik = cdd(0, 1) * cdd((*k_obj)[m->vobj[v]].x, (*k_obj)[m->vobj[v]].y);
            a[v] = d2(ik);
            ai[v] = d2(1.0 / ik);
        }
        st->ikv.upload(a);
        st->iikv.upload(ai);
    }
    // numeric factorisations, one thread per system
    const int nf = np + 2;
    st->nfactors = nf;
    const LdlSymbolic &S = sy.sym;
    const int64_t nnz = S.nnzL();
    std::vector<std::vector<cd>> Ds(nf), Ls(nf), Is(nf), ITs(nf);
    std::vector<int> ok(nf, 0);
    auto factor = [&](int f) {
        // beta of system f: B_j (shifts), 1 (M - S/k_eps^2), 0 (M); times c_i
        cdd beta = f < np ? B[f] : (f == np ? cdd(1.0) : cdd(0.0));
        std::vector<cd> vals(sy.gcol.size());
        for (int i = 0; i < n; i++) {
            const cdd ci = cobj[m->vobj[i]];
            for (int e2 = sy.gptr[i]; e2 < sy.gptr[i + 1]; e2++)
                vals[e2] = sy.Mv[e2] - beta * ci * sy.Sv[e2];
        }
        ok[f] = ldl_numeric(S, vals, Ds[f], Ls[f]) ? 1 : 0;
        if (ok[f]) ldl_block_inverses(S, Ls[f], Is[f], ITs[f]);
    };
    {
        std::vector<std::thread> th;
        for (int f = 0; f < nf; f++) th.emplace_back(factor, f);
        for (auto &t : th) t.join();
    }
    for (int f = 0; f < nf; f++)
        if (!ok[f]) fail(BEM_E_NAN, "zero pivot in OSRC factorisation " + std::to_string(f));
    const int64_t nd = S.ndense;
    std::vector<double2> Dinv((size_t)nf * n), Lc((size_t)nf * nnz), Lr((size_t)nf * nnz);
    std::vector<double2> iL((size_t)nf * nd), iLT((size_t)nf * nd);
    for (int f = 0; f < nf; f++) {
        for (int i = 0; i < n; i++) Dinv[(size_t)f * n + i] = d2(1.0 / Ds[f][i]);
        for (int64_t p = 0; p < nnz; p++) Lc[(size_t)f * nnz + p] = d2(Ls[f][p]);
        for (int64_t p = 0; p < nnz; p++) Lr[(size_t)f * nnz + p] = d2(Ls[f][S.Rmap[p]]);
        for (int64_t p = 0; p < nd; p++) {
            iL[(size_t)f * nd + p] = d2(Is[f][p]);
            iLT[(size_t)f * nd + p] = d2(ITs[f][p]);
        }
    }
    st->Dinv.upload(Dinv);
    st->Lcsc.upload(Lc);
    st->Lcsr.upload(Lr);
    st->invL.upload(iL);
    st->invLT.upload(iLT);
    st->ensure_batch(1);
    (void)s;
    if (m->osrc_cache.size() >= 4) m->osrc_cache.erase(m->osrc_cache.begin());
    auto &ref = *st;
    m->osrc_cache[key] = std::move(st);
    return ref;
}

void osrc_apply_from_weak(bem_mesh *m, OsrcState &st, const double2 *yw, double2 *z, int R,
                          hipStream_t s, const OsrcScratch *scr) {
    OsrcSymbolicState &sy = *m->osrc_sym;
    const int n = sy.n, np = st.np, nt = osrc_tasks(np);
    if (!scr) st.ensure_batch(R);
    const LdlDev L = ldl_view(sy, st);
    const cdd ik = cdd(0, 1) * cdd(st.k.x, st.k.y);
    const double2 one = make_double2(1.0, 0.0);
    // right-hand side r: yw + r 2n in, z + r 2n out, obuf + r os, work + r ws
    const int64_t wl = sy.wlen;
    const int64_t n2 = 2 * (int64_t)n, os = osrc_obuf_len(np, n), ws = (int64_t)nt * wl;
    double2 *ob = scr ? scr->obuf : st.obuf.p, *wk = scr ? scr->work : st.work.p;
    const LdlSplitDev P = split_view(sy, nt, R);
    double2 *u1 = ob + (size_t)np * n;
    Timer tm("osrc_apply", s);
    if (osrc_one_stage(np)) {
        // DtN: shifted solves and M^{-1} on y1; NtD: the same shifts and
        // (M - S/k_eps^2)^{-1} on y2 (R(X)(I + X)^{-1} in partial fractions)
        double2 *s2 = ob + (size_t)(np + 1) * n, *v = ob + (size_t)(2 * np + 1) * n;
        TaskList ta{};
        for (int j = 0; j < np; j++) {
            ta.t[j] = SolveTask{j, yw, ob + (size_t)j * n, one, wk + j * wl};
            ta.t[np + 1 + j] = SolveTask{j, yw + n, s2 + (size_t)j * n, one, wk + (np + 1 + j) * wl};
        }
        ta.t[np] = SolveTask{np + 1, yw, u1, one, wk + np * wl};
        ta.t[2 * np + 1] = SolveTask{np, yw + n, v, one, wk + (2 * np + 1) * wl};
        ta.in_stride = n2;
        ta.out_stride = os;
        ta.work_stride = ws;
        launch_ldl_solve(L, P, ta, nt, R, s);
        // z1 = ik (C_0' u - sum_j (A_j/B_j) s_j);  z2 = (1/ik) (D_0 v + sum_j E_j s'_j)
        launch_pade_pair(n, st.pf, d2(ik), st.ikv.p, u1, os, ob, n, os, z, n2, st.qf,
                         d2(1.0 / ik), st.iikv.p, v, s2, z + n, R, s);
        return;
    }
    double2 *v = ob + (size_t)(np + 1) * n, *m2 = ob + (size_t)(np + 2) * n;
    // stage 1: shifted solves and M^{-1} on y1 (DtN); (M - S/k_eps^2)^{-1} on y2 (NtD)
    TaskList ta{};
    for (int j = 0; j < np; j++) ta.t[j] = SolveTask{j, yw, ob + (size_t)j * n, one, wk + j * wl};
    ta.t[np] = SolveTask{np + 1, yw, u1, one, wk + np * wl};
    ta.t[np + 1] = SolveTask{np, yw + n, v, one, wk + (np + 1) * wl};
    ta.in_stride = n2;
    ta.out_stride = os;
    ta.work_stride = ws;
    launch_ldl_solve(L, P, ta, np + 2, R, s);
    // z1 = ik (C_0' M^{-1} y1 - sum_j (A_j/B_j) s_j);  m2 = M v
    launch_pade_sum_spmv(n, st.pf, d2(ik), st.ikv.p, u1, os, ob, n, os, z, n2, R, sy.gptr_d.p,
                         sy.gcol_d.p, sy.Mv_d.p, v, os, m2, os, R, s);
    // stage 2: shifted solves on M v (NtD)
    TaskList tb{};
    for (int j = 0; j < np; j++) tb.t[j] = SolveTask{j, m2, ob + (size_t)j * n, one, wk + j * wl};
    tb.in_stride = os;
    tb.out_stride = os;
    tb.work_stride = ws;
    launch_ldl_solve(L, P, tb, np, R, s);
    // z2 = (1/ik) (C_0' v - sum_j (A_j/B_j) s'_j)
    launch_pade_sum(n, st.pf, d2(1.0 / ik), st.iikv.p, v, os, ob, n, os, z + n, n2, R, s);
}

void osrc_apply_strong(bem_mesh *m, OsrcState &st, const double2 *x, double2 *y, int R,
                       hipStream_t s, const OsrcScratch *scr) {
    OsrcSymbolicState &sy = *m->osrc_sym;
    if (!scr) st.ensure_batch(R);
    double2 *wb = scr ? scr->wbuf : st.wbuf.p;
    launch_spmv_real(sy.n, 2 * R, sy.gptr_d.p, sy.gcol_d.p, sy.Mv_d.p, x, sy.n, wb, sy.n, s);
    osrc_apply_from_weak(m, st, wb, y, R, s, scr);
}

void osrc_mass_solve(bem_mesh *m, OsrcState &st, const double2 *x, double2 *y, int nblocks,
                     hipStream_t s) {
    OsrcSymbolicState &sy = *m->osrc_sym;
    const int n = sy.n;
    const LdlDev L = ldl_view(sy, st);
    TaskList t{};
    int nb = std::min(nblocks, st.np + 2);
    for (int b0 = 0; b0 < nblocks; b0 += nb) {
        int cnt = std::min(nb, nblocks - b0);
        for (int b = 0; b < cnt; b++)
            t.t[b] = SolveTask{st.np + 1, x + (size_t)(b0 + b) * n, y + (size_t)(b0 + b) * n,
                               make_double2(1.0, 0.0), st.work.p + (size_t)b * sy.wlen};
        launch_ldl_solve(L, split_view(sy, cnt, 1), t, cnt, 1, s);
    }
}

}   // namespace bem

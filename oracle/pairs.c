/*
 * oracle/pairs.c -- FP64 Galerkin pair integrals on flat P1 triangles.
 * TEST INFRASTRUCTURE ONLY: the oracle of the GPU path; plain loops, no
 * blocking, no reordering beyond the quadrature sums themselves.
 *
 * For a test triangle tau (point x, normal n_x) and a trial triangle sigma
 * (point y, normal n_y), with r = |x - y|, the Helmholtz Green's function
 * G = exp(i k r) / (4 pi r) (Sec. 2.2) and F = G (i k r - 1) / r^2
 * (so that grad_x G = F (x - y)), the local 3x3 blocks are
 *
 *   V [a][b] = int int G                      phi_a(x) phi_b(y)
 *   K [a][b] = int int F ((y - x) . n_y)      phi_a(x) phi_b(y)   (d/dn_y G)
 *   Kp[a][b] = int int F ((x - y) . n_x)      phi_a(x) phi_b(y)   (d/dn_x G)
 *   D [a][b] = int int G [curl phi_a . curl phi_b - k^2 (n_x . n_y) phi_a phi_b]
 *
 * D is the hypersingular operator (with the paper's minus sign, Sec. 2.2) in
 * its integrated-by-parts (Maue) form; curl phi = n x grad_Gamma phi.
 *
 * Quadrature: pairs that share no vertex use the 6x6 tensor product of the
 * 6-point triangle rule; coinciding pairs and pairs sharing an edge or a vertex
 * use the singular rules passed in as tables of (x1, x2, y1, y2, w) over the
 * reference triangle K = {0 <= x2 <= x1 <= 1}, chi(x) = A + x1 (B-A) + x2 (C-B).
 * Vertex labelling for the singular rules: coincident: (A,B,C) = local
 * (0,1,2); common edge: A = the shared vertex with the smaller global index,
 * B = the other shared vertex, C = the remaining vertex of each triangle;
 * common vertex: A = the shared vertex, then B, C follow each triangle's own
 * cyclic order.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
    double v[3][3];      /* vertex coordinates */
    int id[3];           /* global vertex ids */
    double n[3];         /* unit normal (v1-v0)x(v2-v0)/|.| */
    double area;
    double curl[3][3];   /* curl phi_a = n x grad phi_a */
} tri_t;

static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void load_tri(const double *P, const int *tri, int t, tri_t *T) {
    for (int a = 0; a < 3; a++) {
        T->id[a] = tri[3 * t + a];
        for (int c = 0; c < 3; c++) T->v[a][c] = P[3 * T->id[a] + c];
    }
    double e1[3], e2[3], nn[3];
    for (int c = 0; c < 3; c++) {
        e1[c] = T->v[1][c] - T->v[0][c];
        e2[c] = T->v[2][c] - T->v[0][c];
    }
    cross3(e1, e2, nn);
    double len = sqrt(dot3(nn, nn));
    T->area = 0.5 * len;
    for (int c = 0; c < 3; c++) T->n[c] = nn[c] / len;
    /* grad phi_a = n x (v_{a+2} - v_{a+1}) / (2|tau|); curl = n x grad */
    for (int a = 0; a < 3; a++) {
        double e[3], g[3];
        for (int c = 0; c < 3; c++)
            e[c] = T->v[(a + 2) % 3][c] - T->v[(a + 1) % 3][c];
        cross3(T->n, e, g);
        for (int c = 0; c < 3; c++) g[c] /= 2.0 * T->area;
        cross3(T->n, g, T->curl[a]);
    }
}

/* local order (A,B,C) -> local vertex indices of the triangle */
static void relabel_vertex(const tri_t *T, int shared, int perm[3]) {
    int a = 0;
    while (T->id[a] != shared) a++;
    perm[0] = a;
    perm[1] = (a + 1) % 3;
    perm[2] = (a + 2) % 3;
}

static void relabel_edge(const tri_t *T, int A, int B, int perm[3]) {
    for (int a = 0; a < 3; a++) {
        if (T->id[a] == A) perm[0] = a;
        else if (T->id[a] == B) perm[1] = a;
        else perm[2] = a;
    }
}

/* Accumulate one quadrature point pair into the four local blocks. */
static void add_point(const tri_t *X, const tri_t *Y, const double *lx,
                      const double *ly, double w, cplx k, cplx blk[4][3][3]) {
    double x[3], y[3], d[3];
    for (int c = 0; c < 3; c++) {
        x[c] = lx[0] * X->v[0][c] + lx[1] * X->v[1][c] + lx[2] * X->v[2][c];
        y[c] = ly[0] * Y->v[0][c] + ly[1] * Y->v[1][c] + ly[2] * Y->v[2][c];
        d[c] = x[c] - y[c];
    }
    double r = sqrt(dot3(d, d));
    cplx G = cexp(I * k * r) / (4.0 * M_PI * r);
    cplx F = G * (I * k * r - 1.0) / (r * r);
    double dny = -dot3(d, Y->n);   /* (y - x) . n_y */
    double dnx = dot3(d, X->n);    /* (x - y) . n_x */
    double nn = dot3(X->n, Y->n);
    for (int a = 0; a < 3; a++) {
        for (int b = 0; b < 3; b++) {
            double pp = lx[a] * ly[b] * w;
            double cc = dot3(X->curl[a], Y->curl[b]);
            blk[0][a][b] += G * pp;
            blk[1][a][b] += F * dny * pp;
            blk[2][a][b] += F * dnx * pp;
            blk[3][a][b] += G * (cc * w - k * k * nn * pp);
        }
    }
}

typedef struct {
    const double *reg;   /* [6][4]: bary0 bary1 bary2 weight */
    const double *tab[3]; /* coincident, edge, vertex: [n][5] */
    int ntab[3];
} rules_t;

static void pair_blocks(const tri_t *X, const tri_t *Y, int same, cplx k,
                        const rules_t *R, cplx blk[4][3][3]) {
    memset(blk, 0, sizeof(cplx) * 36);
    int shared[3], ns = 0;
    if (!same) {
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++)
                if (X->id[a] == Y->id[b]) shared[ns++] = X->id[a];
    }
    if (!same && ns == 0) {
        for (int i = 0; i < 6; i++)
            for (int j = 0; j < 6; j++)
                add_point(X, Y, &R->reg[4 * i], &R->reg[4 * j],
                          X->area * Y->area * R->reg[4 * i + 3] *
                              R->reg[4 * j + 3],
                          k, blk);
        return;
    }
    int px[3], py[3], which;
    if (same) {
        which = 0;
        for (int a = 0; a < 3; a++) px[a] = py[a] = a;
    } else if (ns == 2) {
        which = 1;
        int A = shared[0] < shared[1] ? shared[0] : shared[1];
        int B = shared[0] < shared[1] ? shared[1] : shared[0];
        relabel_edge(X, A, B, px);
        relabel_edge(Y, A, B, py);
    } else {
        which = 2;
        relabel_vertex(X, shared[0], px);
        relabel_vertex(Y, shared[0], py);
    }
    const double *tab = R->tab[which];
    double scale = 4.0 * X->area * Y->area;
    for (int q = 0; q < R->ntab[which]; q++) {
        const double *t = &tab[5 * q];
        double bx[3] = {1.0 - t[0], t[0] - t[1], t[1]};
        double by[3] = {1.0 - t[2], t[2] - t[3], t[3]};
        double lx[3], ly[3];
        for (int a = 0; a < 3; a++) {
            lx[px[a]] = bx[a];
            ly[py[a]] = by[a];
        }
        add_point(X, Y, lx, ly, scale * t[4], k, blk);
    }
}

static int skip_pair(const int *obj, int interior, int t, int s) {
    return interior && obj && obj[t] != obj[s];
}

/*
 * Dense assembly of V, K, K', D (each [nv][nv] complex, interleaved re/im,
 * row = test vertex, column = trial vertex), accumulated into out[4].
 * interior != 0 restricts to pairs of triangles of the same object.
 */
void oracle_assemble_dense(const double *P, int nv, const int *tri, int nt,
                           const int *obj, int interior, double kre, double kim,
                           const double *reg, const double *tab0, int n0,
                           const double *tab1, int n1, const double *tab2, int n2,
                           double *outV, double *outK, double *outKp,
                           double *outD) {
    rules_t R = {reg, {tab0, tab1, tab2}, {n0, n1, n2}};
    cplx k = kre + I * kim;
    cplx *out[4] = {(cplx *)outV, (cplx *)outK, (cplx *)outKp, (cplx *)outD};
    const int chunk = 64;
    cplx *buf = (cplx *)calloc((size_t)chunk * 12 * nv, sizeof(cplx));
    for (int t0 = 0; t0 < nt; t0 += chunk) {
        int t1 = t0 + chunk < nt ? t0 + chunk : nt;
        memset(buf, 0, sizeof(cplx) * (size_t)chunk * 12 * nv);
#pragma omp parallel for schedule(dynamic, 1)
        for (int t = t0; t < t1; t++) {
            tri_t X, Y;
            cplx blk[4][3][3];
            load_tri(P, tri, t, &X);
            cplx *row = buf + (size_t)(t - t0) * 12 * nv;
            for (int s = 0; s < nt; s++) {
                if (skip_pair(obj, interior, t, s)) continue;
                load_tri(P, tri, s, &Y);
                pair_blocks(&X, &Y, t == s, k, &R, blk);
                for (int op = 0; op < 4; op++)
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++)
                            row[(size_t)(op * 3 + a) * nv + Y.id[b]] +=
                                blk[op][a][b];
            }
        }
        for (int t = t0; t < t1; t++) {
            cplx *row = buf + (size_t)(t - t0) * 12 * nv;
            for (int op = 0; op < 4; op++)
                for (int a = 0; a < 3; a++) {
                    cplx *dst = out[op] + (size_t)tri[3 * t + a] * nv;
                    const cplx *src = row + (size_t)(op * 3 + a) * nv;
                    for (int j = 0; j < nv; j++) dst[j] += src[j];
                }
        }
    }
    free(buf);
}

/*
 * Matrix-free rows: for each listed test triangle t and local vertex a,
 *   out[i][op][a] = sum_sigma sum_b blk_op[a][b] * x_op[sigma_b]
 * with x_op = (xV, xK, xKp, xD) complex [nv]; out is [n_test][4][3] complex.
 */
void oracle_matvec_tris(const double *P, int nv, const int *tri, int nt,
                        const int *obj, int interior, double kre, double kim,
                        const double *reg, const double *tab0, int n0,
                        const double *tab1, int n1, const double *tab2, int n2,
                        const int *test, int n_test, const double *xV,
                        const double *xK, const double *xKp, const double *xD,
                        double *out) {
    (void)nv;
    rules_t R = {reg, {tab0, tab1, tab2}, {n0, n1, n2}};
    cplx k = kre + I * kim;
    const cplx *x[4] = {(const cplx *)xV, (const cplx *)xK, (const cplx *)xKp,
                        (const cplx *)xD};
    cplx *o = (cplx *)out;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_test; i++) {
        int t = test[i];
        tri_t X, Y;
        cplx blk[4][3][3];
        cplx acc[4][3];
        memset(acc, 0, sizeof(acc));
        load_tri(P, tri, t, &X);
        for (int s = 0; s < nt; s++) {
            if (skip_pair(obj, interior, t, s)) continue;
            load_tri(P, tri, s, &Y);
            pair_blocks(&X, &Y, t == s, k, &R, blk);
            for (int op = 0; op < 4; op++)
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++)
                        acc[op][a] += blk[op][a][b] * x[op][Y.id[b]];
        }
        memcpy(&o[(size_t)i * 12], acc, sizeof(acc));
    }
}

/*
 * Integral of a kernel over one given pair with a given singular rule, for the
 * quadrature pins: returns sum_q w_q * f(x_q, y_q) * 4|tau||sigma| where
 * f = exp(i k r) / r ^ p (p = 1 or 0).  Triangles given by coordinates.
 */
void oracle_pair_kernel(const double *vx, const double *vy, int which,
                        const double *tab, int ntab, const int *px,
                        const int *py, double kre, double kim, int power,
                        double *res) {
    tri_t X, Y;
    int ids[3] = {0, 1, 2};
    double P[18];
    memcpy(P, vx, 9 * sizeof(double));
    memcpy(P + 9, vy, 9 * sizeof(double));
    int tri[6] = {0, 1, 2, 3, 4, 5};
    load_tri(P, tri, 0, &X);
    load_tri(P, tri, 1, &Y);
    (void)ids;
    (void)which;
    cplx k = kre + I * kim, acc = 0;
    for (int q = 0; q < ntab; q++) {
        const double *t = &tab[5 * q];
        double bx[3] = {1.0 - t[0], t[0] - t[1], t[1]};
        double by[3] = {1.0 - t[2], t[2] - t[3], t[3]};
        double lx[3], ly[3], x[3], y[3], d[3];
        for (int a = 0; a < 3; a++) {
            lx[px[a]] = bx[a];
            ly[py[a]] = by[a];
        }
        for (int c = 0; c < 3; c++) {
            x[c] = lx[0] * X.v[0][c] + lx[1] * X.v[1][c] + lx[2] * X.v[2][c];
            y[c] = ly[0] * Y.v[0][c] + ly[1] * Y.v[1][c] + ly[2] * Y.v[2][c];
            d[c] = x[c] - y[c];
        }
        double r = sqrt(dot3(d, d));
        cplx f = cexp(I * k * r);
        if (power == 1) f /= r;
        acc += t[4] * f;
    }
    acc *= 4.0 * X.area * Y.area;
    res[0] = creal(acc);
    res[1] = cimag(acc);
}

#ifdef _OPENMP
#include <omp.h>
#endif
/* Number of OpenMP threads the oracle's pair loops use. */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

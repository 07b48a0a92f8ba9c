// Quadrature tables: 6-point triangle rule and the singular rules used for
// triangle pairs that coincide or share an edge or a vertex (the Galerkin
// discretisation of Sec. 2.3 integrates weakly singular kernels over such
// pairs; Sauter & Schwab, Boundary Element Methods, Sec. 5.2).
//
// Reference triangle K = {(x1,x2): 0 <= x2 <= x1 <= 1}; a triangle (A,B,C) is
// chi(x) = A + x1 (B-A) + x2 (C-B), barycentrics (1-x1, x1-x2, x2).  Each rule
// is a 4-fold tensor Gauss-Legendre rule on [0,1]^4 pushed through a map built
// from relative coordinates; weights sum to |K|^2 = 1/4:
//  * coincident: z = y - x over the hexagon K - K, six sectors on which
//    g(z) = max(0,z1) + max(0,-z2) + max(0,z2-z1) is linear, z = xi (v_i +
//    eta (v_{i+1} - v_i)); the admissible x form K n (K - z), a copy of K
//    scaled by 1 - xi.  Weight xi (1-xi)^2 alpha.
//  * common edge (A-B shared): w = (y1-x1, x2, y2) scaled radially against
//    the gauge max(z1 + x2, y2) (two faces) and the mirror y1 < x1; the free
//    coordinate spans an interval of length 1 - xi.  Four regions.
//  * common vertex (A shared): x = x1 (1,u), y = y1 (1,v), split at x1 = y1.
#include <cmath>

#include "bem_internal.h"

namespace bem {

namespace {

// Gauss-Legendre nodes/weights on [0,1] by Newton iteration on P_n.
void gauss_legendre01(int n, std::vector<double> &t, std::vector<double> &w) {
    t.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; i++) {
        double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pn = (n == 1) ? x : p1;
            double pm = (n == 1) ? 1.0 : p0;
            dp = n * (x * pn - pm) / (x * x - 1.0);
            double dx = pn / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        // recompute derivative at the converged node
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; k++) {
            double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (x * p1 - p0) / (x * x - 1.0);
        t[n - 1 - i] = 0.5 * (x + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - x * x) * dp * dp);   // 2/((1-x^2)P'^2) / 2
    }
}

void push(std::vector<double> &v, double x1, double x2, double y1, double y2,
          double w) {
    v.push_back(x1);
    v.push_back(x2);
    v.push_back(y1);
    v.push_back(y2);
    v.push_back(w);
}

Rules make_rules() {
    Rules R;
    // Dunavant (1985) degree-4 rule: orbits (1-2a, a, a)
    const double a1 = 0.44594849091596488631832925388305;
    const double w1 = 0.22338158967801146569500700843312;
    const double a2 = 0.091576213509770743459571463402202;
    const double w2 = 0.10995174365532186763832632490021;
    const double orb[2][2] = {{a1, w1}, {a2, w2}};
    int q = 0;
    for (int o = 0; o < 2; o++) {
        double a = orb[o][0], b = 1.0 - 2.0 * a;
        double pts[3][3] = {{b, a, a}, {a, b, a}, {a, a, b}};
        for (int j = 0; j < 3; j++, q++) {
            for (int c = 0; c < 3; c++) R.reg_bary[q][c] = pts[j][c];
            R.reg_w[q] = orb[o][1];
        }
    }

    const int n = 4;
    std::vector<double> t, w;
    gauss_legendre01(n, t, w);

    // coincident
    const double hex[6][2] = {{1, 0}, {1, 1}, {0, 1}, {-1, 0}, {-1, -1}, {0, -1}};
    for (int s = 0; s < 6; s++) {
        const double *v0 = hex[s], *v1 = hex[(s + 1) % 6];
        double jac = std::fabs(v0[0] * (v1[1] - v0[1]) - v0[1] * (v1[0] - v0[0]));
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++)
                for (int k = 0; k < n; k++)
                    for (int l = 0; l < n; l++) {
                        double xi = t[i], eta = t[j], al = t[k], be = t[l];
                        double z1 = xi * (v0[0] + eta * (v1[0] - v0[0]));
                        double z2 = xi * (v0[1] + eta * (v1[1] - v0[1]));
                        double a = std::fmax(0.0, -z2);
                        double b = std::fmax(0.0, z2 - z1);
                        double sc = 1.0 - xi;
                        double x2 = a + sc * al * be;
                        double x1 = x2 + b + sc * al * (1.0 - be);
                        push(R.ss[0], x1, x2, x1 + z1, x2 + z2,
                             w[i] * w[j] * w[k] * w[l] * jac * xi * sc * sc * al);
                    }
    }
    // common edge: faces z1 + x2 = 1 and y2 = 1, then the mirrors
    std::vector<double> e1, e2;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++)
                for (int l = 0; l < n; l++) {
                    double xi = t[i], tt = t[j], u = t[k], v = t[l];
                    double ww = w[i] * w[j] * w[k] * w[l];
                    double L = 1.0 - xi;
                    double y1 = 1.0 - L * tt;
                    double z1 = xi * (1.0 - u);
                    push(e1, y1 - z1, xi * u, y1, xi * v, ww * xi * xi * L);
                    z1 = xi * u * (1.0 - v);
                    push(e2, y1 - z1, xi * u * v, y1, xi, ww * xi * xi * L * u);
                }
    R.ss[1] = e1;
    R.ss[1].insert(R.ss[1].end(), e2.begin(), e2.end());
    for (const std::vector<double> *src : {&e1, &e2})
        for (size_t r = 0; r < src->size(); r += 5)
            push(R.ss[1], (*src)[r + 2], (*src)[r + 3], (*src)[r + 0], (*src)[r + 1],
                 (*src)[r + 4]);
    // common vertex
    std::vector<double> v1;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++)
                for (int l = 0; l < n; l++) {
                    double xi = t[i], eta = t[j], u = t[k], v = t[l];
                    double ww = w[i] * w[j] * w[k] * w[l];
                    push(v1, xi, xi * u, xi * eta, xi * eta * v, ww * xi * xi * xi * eta);
                }
    R.ss[2] = v1;
    for (size_t r = 0; r < v1.size(); r += 5)
        push(R.ss[2], v1[r + 2], v1[r + 3], v1[r + 0], v1[r + 1], v1[r + 4]);
    return R;
}

}   // namespace

const Rules &rules() {
    static const Rules R = make_rules();
    return R;
}

}   // namespace bem

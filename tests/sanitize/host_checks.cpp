// Host-only checks of the mesh validation, the singular and regular
// quadrature rules and the sparse complex-symmetric LDL^T, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host side
// (test_host_sanitizers.py).  Without a GPU, a valid mesh passes validation
// and the geometry set-up and then stops at its first device allocation.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <vector>

#include "bem_internal.h"
#include "osrc_internal.h"
#include "sparse_ldl.h"

// Definitions that live with the library's C entry points and its OSRC and
// compressed-operator sources: the error helpers, the device-memory release
// registry, the mesh handle's destructor and its cache deleters.  The checks build no compressed operator,
// so that deleter never runs.
namespace bem {
[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }
void set_last_error(const std::string &) {}
bool release_device_memory() { return false; }   // no serving caches here
void OsrcDeleter::operator()(OsrcState *p) const { delete p; }
void OsrcSymDeleter::operator()(OsrcSymbolicState *p) const { delete p; }
void HMatDeleter::operator()(HMatrix *) const { std::abort(); }
}   // namespace bem
bem_mesh::~bem_mesh() = default;

namespace {

int failures = 0;
#define CHECK(cond, ...)                                                                        \
    do {                                                                                       \
        if (!(cond)) {                                                                         \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__);                                   \
            std::printf(__VA_ARGS__);                                                          \
            std::printf("\n");                                                                 \
            failures++;                                                                        \
        }                                                                                      \
    } while (0)

// octahedron subdivided `levels` times, vertices on the unit sphere, outward
// counter-clockwise triangles
void sphere(int levels, std::vector<double> &P, std::vector<int32_t> &T) {
    P = {1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1};
    T = {0, 2, 4, 2, 1, 4, 1, 3, 4, 3, 0, 4, 2, 0, 5, 1, 2, 5, 3, 1, 5, 0, 3, 5};
    for (int l = 0; l < levels; l++) {
        std::map<std::pair<int, int>, int> mid;
        auto midpoint = [&](int a, int b) {
            const std::pair<int, int> k(std::min(a, b), std::max(a, b));
            auto it = mid.find(k);
            if (it != mid.end()) return it->second;
            double v[3], n = 0;
            for (int c = 0; c < 3; c++) {
                v[c] = 0.5 * (P[3 * a + c] + P[3 * b + c]);
                n += v[c] * v[c];
            }
            for (int c = 0; c < 3; c++) P.push_back(v[c] / std::sqrt(n));
            const int id = (int)P.size() / 3 - 1;
            mid[k] = id;
            return id;
        };
        std::vector<int32_t> nt;
        for (size_t t = 0; t < T.size(); t += 3) {
            const int a = T[t], b = T[t + 1], c = T[t + 2];
            const int ab = midpoint(a, b), bc = midpoint(b, c), ca = midpoint(c, a);
            for (int v : {a, ab, ca, ab, b, bc, ca, bc, c, ab, bc, ca}) nt.push_back(v);
        }
        T.swap(nt);
    }
}

int build_code(const std::vector<double> &P, const std::vector<int32_t> &T,
               const std::vector<int32_t> *obj = nullptr) {
    bem_mesh m;
    try {
        bem::mesh_build(&m, P.data(), (int64_t)P.size() / 3, T.data(), (int64_t)T.size() / 3,
                        obj ? obj->data() : nullptr);
        return 0;
    } catch (const bem::Error &e) {
        return e.code;
    }
}

void check_quadrature() {
    const bem::Rules &R = bem::rules();
    double ws = 0;
    for (int q = 0; q < 6; q++) {
        ws += R.reg_w[q];
        CHECK(std::fabs(R.reg_bary[q][0] + R.reg_bary[q][1] + R.reg_bary[q][2] - 1) < 1e-15,
              "barycentric row %d", q);
    }
    CHECK(std::fabs(ws - 1) < 1e-14, "regular weights sum %.17g", ws);
    for (int k = 0; k < 3; k++) {
        const std::vector<double> &r = R.ss[k];
        CHECK(!r.empty() && r.size() % 5 == 0, "singular rule %d size", k);
        double w = 0;
        for (size_t i = 0; i < r.size(); i += 5) {
            w += r[i + 4];
            // points in K = {0 <= x2 <= x1 <= 1} for both triangles
            CHECK(r[i + 1] >= -1e-15 && r[i + 1] <= r[i] + 1e-15 && r[i] <= 1 + 1e-15,
                  "rule %d point x", k);
            CHECK(r[i + 3] >= -1e-15 && r[i + 3] <= r[i + 2] + 1e-15 && r[i + 2] <= 1 + 1e-15,
                  "rule %d point y", k);
        }
        CHECK(std::fabs(w - 0.25) < 1e-13, "singular rule %d weight sum %.17g (|K|^2 = 1/4)", k, w);
    }
}

void check_mesh() {
    std::vector<double> P;
    std::vector<int32_t> T;
    sphere(3, P, T);
    const int ok = build_code(P, T);
    // valid: built (GPU present) or stopped at the first device allocation
    CHECK(ok == 0 || ok == BEM_E_NOMEM || ok == BEM_E_DEVICE, "valid mesh: code %d", ok);
    std::printf("valid mesh of %zu vertices: code %d\n", P.size() / 3, ok);
    {   // open surface
        std::vector<int32_t> t2(T.begin(), T.end() - 3);
        CHECK(build_code(P, t2) == BEM_E_BAD_MESH, "open mesh");
    }
    {   // one triangle flipped
        std::vector<int32_t> t2 = T;
        std::swap(t2[1], t2[2]);
        CHECK(build_code(P, t2) == BEM_E_BAD_MESH, "flipped triangle");
    }
    {   // all triangles flipped: inward normals
        std::vector<int32_t> t2 = T;
        for (size_t t = 0; t < t2.size(); t += 3) std::swap(t2[t + 1], t2[t + 2]);
        CHECK(build_code(P, t2) == BEM_E_BAD_MESH, "inward normals");
    }
    {   // index out of range
        std::vector<int32_t> t2 = T;
        t2[7] = (int32_t)(P.size() / 3);
        CHECK(build_code(P, t2) == BEM_E_INVAL, "index out of range");
    }
    {   // non-finite vertex
        std::vector<double> p2 = P;
        p2[4] = NAN;
        CHECK(build_code(p2, T) == BEM_E_INVAL, "NaN vertex");
    }
    {   // two objects sharing vertices
        std::vector<int32_t> obj(T.size() / 3, 0);
        obj[0] = 1;
        CHECK(build_code(P, T, &obj) == BEM_E_BAD_MESH, "objects sharing a vertex");
    }
    {   // too few triangles
        std::vector<int32_t> t2(T.begin(), T.begin() + 9);
        CHECK(build_code(P, t2) == BEM_E_INVAL, "three triangles");
    }
}

// A = (c I + L) (1 + 0.3 i) on the vertex graph of the sphere, L its graph
// Laplacian: complex symmetric with a nonsingular real part
void check_ldl() {
    std::vector<double> P;
    std::vector<int32_t> T;
    sphere(4, P, T);
    const int n = (int)P.size() / 3;
    std::vector<std::vector<int32_t>> nb(n);
    for (size_t t = 0; t < T.size(); t += 3)
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++)
                if (a != b) nb[T[t + a]].push_back(T[t + b]);
    std::vector<int32_t> ptr(1, 0), col;
    for (int i = 0; i < n; i++) {
        nb[i].push_back(i);
        std::sort(nb[i].begin(), nb[i].end());
        nb[i].erase(std::unique(nb[i].begin(), nb[i].end()), nb[i].end());
        col.insert(col.end(), nb[i].begin(), nb[i].end());
        ptr.push_back((int32_t)col.size());
    }
    const bem::cd s(1.0, 0.3);
    std::vector<bem::cd> vals(col.size());
    for (int i = 0; i < n; i++)
        for (int e = ptr[i]; e < ptr[i + 1]; e++)
            vals[e] = (col[e] == i ? bem::cd(0.5 + (ptr[i + 1] - ptr[i] - 1), 0) : bem::cd(-1, 0)) * s;
    const std::vector<int32_t> group(n, 0);
    for (int leaf : {8, 48}) {
        const bem::NdOrder nd = bem::nested_dissection(n, ptr, col, P, group, leaf);
        const bem::LdlSymbolic S = bem::ldl_symbolic(n, ptr, col, nd);
        std::vector<bem::cd> D, Lx, iL, iLT;
        CHECK(bem::ldl_numeric(S, vals, D, Lx), "zero pivot");
        bem::ldl_block_inverses(S, Lx, iL, iLT);
        std::vector<bem::cd> b(n), x0, x1, x2;
        for (int i = 0; i < n; i++) b[i] = bem::cd(std::sin(0.1 * i), std::cos(0.37 * i));
        bem::ldl_solve_host(S, D, Lx, b, x0);
        bem::ldl_solve_blocks_host(S, D, Lx, iL, iLT, b, x1);
        double rn = 0, bn = 0, d1 = 0;
        for (int i = 0; i < n; i++) {
            bem::cd r = b[i];
            for (int e = ptr[i]; e < ptr[i + 1]; e++) r -= vals[e] * x0[col[e]];
            rn += std::norm(r);
            bn += std::norm(b[i]);
            d1 += std::norm(x1[i] - x0[i]);
        }
        CHECK(std::sqrt(rn / bn) < 1e-12, "LDL residual %.3g (leaf %d)", std::sqrt(rn / bn), leaf);
        CHECK(std::sqrt(d1 / bn) < 1e-12, "block solve differs %.3g (leaf %d)", std::sqrt(d1 / bn), leaf);
        for (int sub : {64, 256, 1 << 20}) {
            const bem::LdlSplit sp = bem::ldl_split_plan(S, sub, 1 << 20, 1 << 20);
            if (!sp.ok) continue;
            bem::ldl_solve_split_host(S, sp, D, Lx, iL, iLT, b, x2);
            double d2 = 0;
            for (int i = 0; i < n; i++) d2 += std::norm(x2[i] - x0[i]);
            CHECK(std::sqrt(d2 / bn) < 1e-12, "split solve differs %.3g (leaf %d, sub %d)",
                  std::sqrt(d2 / bn), leaf, sub);
        }
    }
}

}   // namespace

int main() {
    check_quadrature();
    check_mesh();
    check_ldl();
    std::printf("host checks: %d failures\n", failures);
    return failures ? 1 : 0;
}

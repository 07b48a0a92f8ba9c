// Autotuner: times the launch choices of the operator for one mesh size and
// right-hand-side count on the device (pair-kernel workgroup size and vectors
// per launch; matrix-free against the assembled complex64 operator with its
// product kernel) and keeps the fastest in a table keyed by (triangles,
// right-hand-side bucket), optionally persisted in a text file, one entry
// per line:
//   bem-tune-v1 <arch> T=<triangles> R=<bucket> block=<b> multi=<m>
//       gemm_min=<g> [skinny_min=<s>] path=<p> t_mf=<s> t_dense=<s> t_asm=<s>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "bem_internal.h"

namespace bem {

namespace {

std::mutex g_mu;
std::map<std::pair<int64_t, int>, TuneEntry> g_table;
std::string g_cache_path, g_cache_arch;

std::string device_arch() {
    int dev = 0;
    BEM_HIP(hipGetDevice(&dev));
    hipDeviceProp_t p;
    BEM_HIP(hipGetDeviceProperties(&p, dev));
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

std::string format_entry(const std::string &arch, int64_t T, int R, const TuneEntry &e) {
    char buf[512];
    std::snprintf(buf, sizeof(buf),
                  "bem-tune-v1 %s T=%lld R=%d block=%d multi=%d gemm_min=%d skinny_min=%d "
                  "path=%d t_mf=%.9g t_dense=%.9g t_asm=%.9g",
                  arch.c_str(), (long long)T, R, e.block, e.multi, e.gemm_min, e.skinny_min,
                  e.path, e.t_mf, e.t_dense, e.t_asm);
    return buf;
}

// Parses one line; false if malformed or for another architecture.
bool parse_entry(const std::string &line, const std::string &arch, int64_t &T, int &R,
                 TuneEntry &e) {
    std::istringstream in(line);
    std::string tag, a;
    if (!(in >> tag >> a) || tag != "bem-tune-v1" || a != arch) return false;
    std::map<std::string, std::string> kv;
    std::string tok;
    while (in >> tok) {
        const size_t eq = tok.find('=');
        if (eq == std::string::npos) return false;
        kv[tok.substr(0, eq)] = tok.substr(eq + 1);
    }
    try {
        T = std::stoll(kv.at("T"));
        R = std::stoi(kv.at("R"));
        e.block = std::stoi(kv.at("block"));
        e.multi = std::stoi(kv.at("multi"));
        e.gemm_min = std::stoi(kv.at("gemm_min"));
        if (kv.count("skinny_min")) e.skinny_min = std::stoi(kv.at("skinny_min"));
        e.path = std::stoi(kv.at("path"));
        e.t_mf = std::stod(kv.at("t_mf"));
        e.t_dense = std::stod(kv.at("t_dense"));
        e.t_asm = std::stod(kv.at("t_asm"));
    } catch (...) {
        return false;
    }
    return T > 0 && R == tune_bucket(R) && (e.block == 64 || e.block == 128 || e.block == 256) &&
           (e.multi == 1 || e.multi == 2 || e.multi == 4) && e.gemm_min >= 1 && e.skinny_min >= 2 &&
           e.path >= -1 && e.path <= 1;
}

double elapsed_s(hipEvent_t a, hipEvent_t b) {
    float ms = 0;
    BEM_HIP(hipEventSynchronize(b));
    BEM_HIP(hipEventElapsedTime(&ms, a, b));
    return ms * 1e-3;
}

// Best of `reps` timed calls after one warm-up.
template <class F> double time_best(F &&f, hipStream_t s, int reps = 2) {
    hipEvent_t a, b;
    BEM_HIP(hipEventCreate(&a));
    BEM_HIP(hipEventCreate(&b));
    double best = 1e300;
    try {
        f();
        for (int i = 0; i < reps; i++) {
            BEM_HIP(hipEventRecord(a, s));
            f();
            BEM_HIP(hipEventRecord(b, s));
            best = std::min(best, elapsed_s(a, b));
        }
    } catch (...) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        throw;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

}   // namespace

int tune_bucket(int R) { return R >= 16 ? 16 : R >= 8 ? 8 : R >= 4 ? 4 : R >= 2 ? 2 : 1; }

bool tune_find(int64_t T, int R, TuneEntry *e) {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_table.find({T, tune_bucket(R)});
    if (it == g_table.end()) return false;
    if (e) *e = it->second;
    return true;
}

TuneEntry tune_lookup(int64_t T, int R) {
    TuneEntry e;
    if (tune_find(T, R, &e)) return e;
    const Tuning &t = tuning();
    e.block = t.farfield_block;
    e.multi = t.farfield_multi_max;
    e.gemm_min = t.dense_gemm_min_rhs;
    e.skinny_min = t.dense_skinny_min_rhs;
    return e;
}

void tune_store(int64_t T, int R, const TuneEntry &e) {
    std::lock_guard<std::mutex> g(g_mu);
    g_table[{T, tune_bucket(R)}] = e;
    if (!g_cache_path.empty()) {
        std::ofstream out(g_cache_path, std::ios::app);
        if (out) out << format_entry(g_cache_arch, T, tune_bucket(R), e) << "\n";
    }
}

int tune_cache_load(const std::string &path, const std::string &arch) {
    std::ifstream in(path);
    int n = 0;
    std::lock_guard<std::mutex> g(g_mu);
    g_cache_path = path;
    g_cache_arch = arch;
    if (!in) return 0;   // a new cache file: nothing to load
    std::string line;
    while (std::getline(in, line)) {
        int64_t T;
        int R;
        TuneEntry e;
        if (!parse_entry(line, arch, T, R, e)) continue;
        g_table[{T, R}] = e;   // later lines win
        n++;
    }
    return n;
}

void tune_clear() {
    std::lock_guard<std::mutex> g(g_mu);
    g_table.clear();
    g_cache_path.clear();
    g_cache_arch.clear();
}

// Measures and stores the best launch parameters for this mesh and R.
TuneEntry autotune(bem_mesh *m, double2 k0, double2 k1, double rho, int R, int expected,
                   hipStream_t s) {
    const int64_t n2 = 2 * m->N;
    const NearOperator &nf = nearfield_get(m, k0, k1, rho, s);
    DevBuf<double2> X((size_t)R * n2), Y((size_t)R * n2);
    // any finite input: the work does not depend on the values
    BEM_HIP(hipMemsetAsync(X.p, 0, (size_t)R * n2 * sizeof(double2), s));
    TuneEntry best = tune_lookup(m->T, R);
    best.t_mf = 1e300;
    for (int blk : {64, 128, 256})
        for (int mm : {1, 2, 4}) {
            if (mm > 1 && mm > R) continue;
            TuneEntry c = best;
            c.block = blk;
            c.multi = mm;
            const double t = time_best(
                [&] { farfield_apply_batch(m, nf, k0, k1, rho, X.p, Y.p, R, BEM_FP32, s, &c); },
                s);
            if (t < best.t_mf) {
                best.t_mf = t;
                best.block = blk;
                best.multi = mm;
            }
        }
    // assembled operator, when it fits with room to spare
    best.path = 0;
    best.t_dense = best.t_asm = 0;
    size_t free_b = 0, total_b = 0;
    BEM_HIP(hipMemGetInfo(&free_b, &total_b));
    const int64_t need = dense_bytes(m) + dense_assembly_scratch_bytes(m) +
                         dense_gemm_scratch_bytes(m, R) + (2ll << 30);
    if (need < (int64_t)free_b) {
        const auto t0 = std::chrono::steady_clock::now();
        std::unique_ptr<DenseOperator> op = dense_assemble(m, nf, k0, k1, rho, s);
        BEM_HIP(hipStreamSynchronize(s));
        best.t_asm = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        DevBuf<float2> xs;
        TuneEntry c = best;
        c.gemm_min = R + 1;   // multi-vector GEMV
        c.skinny_min = R + 1;
        const double t_gemv = time_best([&] { dense_apply(*op, X.p, Y.p, R, xs, s, &c); }, s);
        double t_skinny = 1e300, t_gemm = 1e300;
        if (R >= 2) {
            c.skinny_min = 2;   // skinny MFMA product
            t_skinny = time_best([&] { dense_apply(*op, X.p, Y.p, R, xs, s, &c); }, s);
            c.gemm_min = R;     // MFMA GEMM
            t_gemm = time_best([&] { dense_apply(*op, X.p, Y.p, R, xs, s, &c); }, s);
        }
        // the whole bucket [b, 2b) takes the faster product
        const int b = tune_bucket(R);
        const double t_small = std::min(t_gemv, t_skinny);
        best.gemm_min = t_gemm < t_small ? b : 2 * b;
        best.skinny_min = t_skinny < t_gemv ? std::max(2, b) : 2 * b;
        best.t_dense = std::min(t_small, t_gemm);
        const double E = std::max(1, expected);
        best.path = best.t_asm + E * best.t_dense < E * best.t_mf ? 1 : 0;
    }
    tune_store(m->T, R, best);
    return best;
}

}   // namespace bem

using bem::fail;

namespace {

void to_c(const bem::TuneEntry &e, bem_tune_entry *o) {
    o->block = e.block;
    o->multi = e.multi;
    o->gemm_min = e.gemm_min;
    o->skinny_min = e.skinny_min;
    o->path = e.path;
    o->t_matrix_free = e.t_mf;
    o->t_assembled = e.t_dense;
    o->t_assembly = e.t_asm;
}

}   // namespace

extern "C" {

int bem_autotune(const bem_mesh *mesh, bem_c64 k_ext, bem_c64 k_int, double rho, int n_rhs,
                 int expected_matvecs, bem_tune_entry *out, void *hip_stream) {
    try {
        if (!mesh) fail(BEM_E_INVAL, "mesh is NULL");
        if (n_rhs < 1 || n_rhs > 64) fail(BEM_E_INVAL, "n_rhs must be in 1..64");
        for (bem_c64 k : {k_ext, k_int})
            if (!std::isfinite(k.re) || !std::isfinite(k.im) || k.im < 0 || (k.re == 0 && k.im == 0))
                fail(BEM_E_INVAL, "wavenumbers must be finite, nonzero, Im k >= 0");
        if (!(rho > 0) || !std::isfinite(rho)) fail(BEM_E_INVAL, "rho must be positive");
        const bem::TuneEntry e = bem::autotune(
            const_cast<bem_mesh *>(mesh), make_double2(k_ext.re, k_ext.im),
            make_double2(k_int.re, k_int.im), rho, n_rhs, expected_matvecs, (hipStream_t)hip_stream);
        if (out) to_c(e, out);
        return BEM_OK;
    } catch (const bem::Error &e) {
        bem::set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        bem::set_last_error("host allocation failed");
        return BEM_E_NOMEM;
    }
}

int bem_tune_cache_load(const char *path, const char *arch, int *n_loaded) {
    try {
        if (!path) fail(BEM_E_INVAL, "path is NULL");
        const std::string a = arch ? std::string(arch) : bem::device_arch();
        const int n = bem::tune_cache_load(path, a);
        if (n_loaded) *n_loaded = n;
        return BEM_OK;
    } catch (const bem::Error &e) {
        bem::set_last_error(e.msg);
        return e.code;
    }
}

int bem_tune_lookup(int64_t n_triangles, int n_rhs, bem_tune_entry *out) {
    if (!out || n_triangles < 1 || n_rhs < 1) {
        bem::set_last_error("bad lookup arguments");
        return BEM_E_INVAL;
    }
    bem::TuneEntry e;
    const bool found = bem::tune_find(n_triangles, n_rhs, &e);
    to_c(found ? e : bem::tune_lookup(n_triangles, n_rhs), out);
    return found ? BEM_OK : BEM_W_DEFAULT;
}

void bem_tune_clear(void) { bem::tune_clear(); }

}   // extern "C"

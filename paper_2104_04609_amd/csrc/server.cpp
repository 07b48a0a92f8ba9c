// Serving loop: queued solve requests, admission by a device-memory budget,
// a pool of worker threads with one HIP stream each, and device-resident mesh
// handles (geometry, near-field, OSRC and dense-operator caches) that persist
// between requests.  Contract and policy are stated in bem.h.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "bem_internal.h"

namespace bem {

namespace {

using Clock = std::chrono::steady_clock;

constexpr double AGED_S = 2.0;            // after this wait, requests go in arrival order
constexpr double HEAD_BLOCK_S = 10.0;     // after this wait, the oldest request blocks others

struct Replica {
    bem_mesh *h = nullptr;    // created lazily by the worker that first runs on it
    bool busy = false;
    int64_t resident = 0;     // device bytes of h while idle
    uint64_t last_used = 0;   // admission tick
};

struct MeshEntry {
    std::shared_ptr<DenseShare> share = std::make_shared<DenseShare>();   // assembled operators
    std::vector<double> P;
    std::vector<int32_t> tri, obj;
    bool has_obj = false;
    int64_t nv = 0, nt = 0;
    int64_t base_bytes = 0;   // a fresh handle after the OSRC symbolic analysis
    std::vector<std::unique_ptr<Replica>> reps;
};

struct Request {
    int64_t id = 0;
    int mesh = 0;
    double2 k0{}, k1{};
    double rho = 0, tol = 0;
    bool per_object = false;   // om holds a material per object
    ObjMaterials om;
    std::vector<double> dirs;
    int n_waves = 0;
    bem_solve_opts o{};
    double2 *solution = nullptr;
    bem_solve_info *info = nullptr;
    int64_t footprint = 0;    // solve footprint (without creating a handle)
    double work = 0;          // admission order: estimated device work
    int64_t reserved = 0;     // footprint + handle creation when admitted
    Replica *rep = nullptr;
    int replica = -1;
    double t_submit = 0, t_admit = 0, t_end = 0;
    int status = BEM_OK;
    std::string msg;
    bool done = false;
};

void destroy_handle(bem_mesh *h) { delete h; }

bem_mesh *create_handle(const MeshEntry &me) {
    std::unique_ptr<bem_mesh> m(new bem_mesh());
    mesh_build(m.get(), me.P.data(), me.nv, me.tri.data(), me.nt,
               me.has_obj ? me.obj.data() : nullptr);
    osrc_prepare(m.get());
    m->dense_share = me.share;
    return m.release();
}

}   // namespace

}   // namespace bem

struct bem_server {
    bem_server_opts o{};
    int device = 0;
    bem::Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<bem::Request>> queue;
    std::map<int64_t, std::shared_ptr<bem::Request>> reqs;
    std::vector<std::unique_ptr<bem::MeshEntry>> meshes;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> threads;
    bool stop = false;
    int64_t next_id = 1;
    uint64_t tick = 0;
    int64_t reserved = 0, peak = 0;
    int inflight = 0, peak_inflight = 0;
    int64_t completed = 0, rejected = 0, evictions = 0;
    int64_t grown = 0;   // Krylov growth reported by running requests (bytes, total)

    double now() const {
        return std::chrono::duration<double>(bem::Clock::now() - t0).count();
    }
    // Cached state of the handles counted against the budget.  Assembled
    // operators that no request holds are a cache outside it: a new request's
    // operator reuses their buffers, and a device allocation that fails
    // releases them (release_hook); those in use are in running footprints.
    int64_t resident() const {
        int64_t b = 0;
        for (const auto &me : meshes)
            for (const auto &r : me->reps) b += r->resident;
        return b;
    }
    // Drops the least recently used assembled operator no request holds (lock
    // held); false if there is none.
    bool evict_shared_op() {
        bem::DenseShare *oldest = nullptr;
        uint64_t t_old = UINT64_MAX;
        for (auto &me : meshes) {
            const uint64_t t = me->share->oldest_idle();
            if (t < t_old) {
                t_old = t;
                oldest = me->share.get();
            }
        }
        if (oldest && oldest->evict_idle_lru() > 0) {
            evictions++;
            return true;
        }
        return false;
    }
    // Releases the cached state of the least recently used idle handle (lock
    // held); false if there is none.
    bool trim_idle_handle() {
        bem::Replica *lru = nullptr;
        bem::MeshEntry *lru_mesh = nullptr;
        for (auto &me : meshes)
            for (auto &r : me->reps)
                if (!r->busy && r->h && r->resident > me->base_bytes &&
                    (!lru || r->last_used < lru->last_used)) {
                    lru = r.get();
                    lru_mesh = me.get();
                }
        if (!lru) return false;
        bem::mesh_trim(lru->h);
        lru->resident = std::max(lru->h->device_bytes(), lru_mesh->base_bytes);
        evictions++;
        return true;
    }
    // A device allocation failed: free an idle assembled operator, else an
    // idle handle's caches.
    static bool release_hook(void *ctx) {
        bem_server *srv = static_cast<bem_server *>(ctx);
        std::lock_guard<std::mutex> g(srv->mu);
        return srv->evict_shared_op() || srv->trim_idle_handle();
    }
    // Release cached state of idle handles, least recently used first, until
    // `need` more bytes fit.  Returns whether they fit.
    bool make_room(int64_t need) {
        while (resident() + reserved + need > o.hbm_budget) {
            if (trim_idle_handle()) continue;
            return false;
        }
        return true;
    }
    // Bytes that stay resident on an otherwise idle server (fresh handles).
    int64_t floor_bytes() const {
        int64_t b = 0;
        for (const auto &me : meshes)
            for (const auto &r : me->reps)
                if (r->h) b += me->base_bytes;
        return b;
    }
    void finish(const std::shared_ptr<bem::Request> &r) {
        r->done = true;
        r->t_end = now();
        cv_done.notify_all();
    }
    // Next admissible request (lock held), or null.  Rejects requests that
    // can never fit.  Order: requests that have waited more than AGED_S in
    // arrival order, then the others smallest estimated work first; once the
    // oldest has waited HEAD_BLOCK_S, no other starts while it does not fit.
    std::shared_ptr<bem::Request> admit() {
        const double t = now();
        std::vector<size_t> order(queue.size());
        for (size_t i = 0; i < order.size(); i++) order[i] = i;
        const bool head_due = !queue.empty() && t - queue.front()->t_submit > bem::HEAD_BLOCK_S;
        std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
            const bool aa = t - queue[a]->t_submit > bem::AGED_S;
            const bool ab = t - queue[b]->t_submit > bem::AGED_S;
            if (aa != ab) return aa;
            if (aa) return false;   // both aged: arrival order (stable)
            return queue[a]->work < queue[b]->work;
        });
        for (size_t oi = 0; oi < order.size();) {
            if (head_due && oi > 0) break;
            const size_t qi = order[oi];
            auto r = queue[qi];
            bem::MeshEntry &me = *meshes[r->mesh];
            bem::Replica *pick = nullptr;
            int pick_i = -1;
            for (size_t i = 0; i < me.reps.size(); i++) {
                bem::Replica *c = me.reps[i].get();
                if (c->busy) continue;
                if (!pick || (c->h && !pick->h) ||
                    ((c->h != nullptr) == (pick->h != nullptr) && c->last_used > pick->last_used)) {
                    pick = c;
                    pick_i = (int)i;
                }
            }
            const bool grow = !pick && (int)me.reps.size() < o.max_replicas;
            if (!pick && !grow) {
                oi++;
                continue;
            }
            const bool fresh = grow || !pick->h;
            const int64_t need = r->footprint + (fresh ? me.base_bytes : 0);
            if (!make_room(need)) {
                if (inflight == 0 && floor_bytes() + need > o.hbm_budget) {
                    r->status = BEM_E_NOMEM;
                    r->msg = "request footprint of " + std::to_string(need) +
                             " bytes exceeds the server budget of " +
                             std::to_string(o.hbm_budget) + " bytes";
                    rejected++;
                    queue.erase(queue.begin() + (long)qi);
                    finish(r);
                    return admit();   // indices changed
                }
                oi++;
                continue;
            }
            if (grow) {
                me.reps.push_back(std::make_unique<bem::Replica>());
                pick = me.reps.back().get();
                pick_i = (int)me.reps.size() - 1;
            }
            pick->busy = true;
            pick->last_used = ++tick;
            r->rep = pick;
            r->replica = pick_i;
            r->reserved = need;
            r->t_admit = t;
            reserved += need;
            inflight++;
            peak_inflight = std::max(peak_inflight, inflight);
            peak = std::max(peak, resident() + reserved);
            queue.erase(queue.begin() + (long)qi);
            return r;
        }
        return nullptr;
    }

    // Growth of a running request's device memory (its Krylov basis) beyond
    // its admission footprint: accounted, with room made from idle caches.
    struct Growth {
        bem_server *srv;
        bem::Request *r;
    };
    static void grow_hook(void *ctx, int64_t delta) {
        Growth *g = static_cast<Growth *>(ctx);
        std::lock_guard<std::mutex> lk(g->srv->mu);
        g->r->reserved += delta;
        g->srv->reserved += delta;
        if (delta > 0) {
            g->srv->grown += delta;
            (void)g->srv->make_room(0);   // over the budget: runs on (bounded by maxiter)
            g->srv->peak = std::max(g->srv->peak, g->srv->resident() + g->srv->reserved);
        }
    }

    void worker(int wi) {
        (void)hipSetDevice(device);
        hipStream_t s = streams[wi];
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            std::shared_ptr<bem::Request> r;
            while (!stop && !(r = admit()))
                cv_work.wait_for(lk, std::chrono::milliseconds(50));
            if (!r) return;
            bem::MeshEntry &me = *meshes[r->mesh];
            bem::Replica *rep = r->rep;
            lk.unlock();
            int status = BEM_OK;
            std::string msg;
            int64_t res = 0;
            try {
                if (!rep->h) rep->h = bem::create_handle(me);
                Growth g{this, r.get()};
                const bem::ReserveScope grow(&bem_server::grow_hook, &g);
                status = bem::solve_run(rep->h, r->k0, r->k1, r->rho, r->dirs.data(), r->n_waves,
                                        r->tol, r->o, r->solution, r->info, s,
                                        r->per_object ? &r->om : nullptr);
            } catch (const bem::Error &e) {
                status = e.code;
                msg = e.msg;
            } catch (const std::bad_alloc &) {
                status = BEM_E_NOMEM;
                msg = "host allocation failed";
            } catch (const std::exception &e) {
                status = BEM_E_DEVICE;
                msg = e.what();
            }
            if (status < 0) (void)hipStreamSynchronize(s);
            if (rep->h) res = std::max(rep->h->device_bytes(), me.base_bytes);
            lk.lock();
            rep->busy = false;
            rep->resident = res;
            rep->last_used = ++tick;
            reserved -= r->reserved;
            inflight--;
            completed++;
            r->status = status;
            r->msg = msg;
            finish(r);
            cv_work.notify_all();
        }
    }
};

using bem::fail;

extern "C" {

void bem_server_opts_default(bem_server_opts *o) {
    if (!o) return;
    o->hbm_budget = 0;
    o->workers = 4;
    o->max_replicas = 0;
    o->dense_max_bytes = -1;
}

int bem_server_create(const bem_server_opts *opts, bem_server **out) {
    try {
        if (!out) fail(BEM_E_INVAL, "out is NULL");
        *out = nullptr;
        std::unique_ptr<bem_server> srv(new bem_server());
        bem_server_opts_default(&srv->o);
        if (opts) srv->o = *opts;
        bem_server_opts &o = srv->o;
        if (o.workers <= 0) o.workers = 4;
        if (o.workers > 64) fail(BEM_E_INVAL, "workers must be at most 64");
        if (o.max_replicas <= 0) o.max_replicas = o.workers;
        if (o.dense_max_bytes < 0) o.dense_max_bytes = 16ll << 30;
        BEM_HIP(hipGetDevice(&srv->device));
        if (o.hbm_budget <= 0) {
            size_t free_b = 0, total_b = 0;
            BEM_HIP(hipMemGetInfo(&free_b, &total_b));
            o.hbm_budget = (int64_t)(0.9 * (double)free_b);
        }
        srv->t0 = bem::Clock::now();
        for (int i = 0; i < o.workers; i++) {
            hipStream_t s = nullptr;
            BEM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            srv->streams.push_back(s);
        }
        bem_server *raw = srv.get();
        bem::add_mem_releaser(&bem_server::release_hook, raw);
        for (int i = 0; i < o.workers; i++) srv->threads.emplace_back([raw, i] { raw->worker(i); });
        *out = srv.release();
        return BEM_OK;
    } catch (const bem::Error &e) {
        bem::set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        bem::set_last_error("host allocation failed");
        return BEM_E_NOMEM;
    }
}

void bem_server_destroy(bem_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->stop = true;
        for (auto &r : srv->queue) {
            r->status = BEM_E_INVAL;
            r->msg = "server shut down";
            srv->finish(r);
        }
        srv->queue.clear();
    }
    srv->cv_work.notify_all();
    for (auto &t : srv->threads) t.join();
    bem::remove_mem_releaser(srv);
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(srv->device);
    for (auto &me : srv->meshes)
        for (auto &r : me->reps) bem::destroy_handle(r->h);
    for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
    (void)hipSetDevice(prev);
    delete srv;
}

int bem_server_add_mesh(bem_server *srv, const double *vertices, int64_t n_vertices,
                        const int32_t *triangles, int64_t n_triangles,
                        const int32_t *object_id, int *mesh_id) {
    int prev = -1;
    try {
        if (!srv || !mesh_id) fail(BEM_E_INVAL, "server or mesh_id is NULL");
        if (!vertices || !triangles || n_vertices < 3 || n_triangles < 4)
            fail(BEM_E_INVAL, "bad mesh arrays");
        auto me = std::make_unique<bem::MeshEntry>();
        me->P.assign(vertices, vertices + 3 * n_vertices);
        me->tri.assign(triangles, triangles + 3 * n_triangles);
        me->has_obj = object_id != nullptr;
        if (object_id) me->obj.assign(object_id, object_id + n_triangles);
        me->nv = n_vertices;
        me->nt = n_triangles;
        BEM_HIP(hipGetDevice(&prev));
        BEM_HIP(hipSetDevice(srv->device));
        auto rep = std::make_unique<bem::Replica>();
        rep->h = bem::create_handle(*me);
        me->base_bytes = rep->h->device_bytes();
        rep->resident = me->base_bytes;
        me->reps.push_back(std::move(rep));
        (void)hipSetDevice(prev);
        prev = -1;
        std::lock_guard<std::mutex> g(srv->mu);
        srv->meshes.push_back(std::move(me));
        *mesh_id = (int)srv->meshes.size() - 1;
        return BEM_OK;
    } catch (const bem::Error &e) {
        if (prev >= 0) (void)hipSetDevice(prev);
        bem::set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        if (prev >= 0) (void)hipSetDevice(prev);
        bem::set_last_error("host allocation failed");
        return BEM_E_NOMEM;
    }
}

namespace {

int server_submit(bem_server *srv, int mesh_id, bem_c64 k_ext, bem_c64 k_int, double rho,
                  const bem_c64 *k_obj, const double *rho_obj, const double *directions,
                  int n_waves, double tol, const bem_solve_opts *opts, bem_c64 *solution,
                  bem_solve_info *info, int64_t *request_id) {
    int prev = -1;
    try {
        if (!srv || !request_id) fail(BEM_E_INVAL, "server or request_id is NULL");
        if (!solution) fail(BEM_E_INVAL, "solution is NULL");
        bem::MeshEntry *me = nullptr;
        bem_mesh *h0 = nullptr;
        {
            std::lock_guard<std::mutex> g(srv->mu);
            if (srv->stop) fail(BEM_E_INVAL, "server is shutting down");
            if (mesh_id < 0 || mesh_id >= (int)srv->meshes.size()) fail(BEM_E_INVAL, "mesh_id");
            me = srv->meshes[mesh_id].get();
            h0 = me->reps[0]->h;   // replica 0 is never released; its sizes are immutable
        }
        auto r = std::make_shared<bem::Request>();
        r->mesh = mesh_id;
        r->k0 = make_double2(k_ext.re, k_ext.im);
        r->k1 = make_double2(k_int.re, k_int.im);
        r->rho = rho;
        r->tol = tol;
        r->n_waves = n_waves;
        bem_solve_opts_default(&r->o);
        if (opts) r->o = *opts;
        bem::solve_check(h0, r->k0, r->k1, rho, directions, n_waves, tol, r->o);
        if (k_obj) {
            if (!rho_obj) fail(BEM_E_INVAL, "rho is NULL");
            r->per_object = true;
            for (int ob = 0; ob < h0->nobj; ob++) {
                r->om.k.push_back(make_double2(k_obj[ob].re, k_obj[ob].im));
                r->om.rho.push_back(rho_obj[ob]);
            }
            bem::check_materials(h0, r->om);
        }
        r->dirs.assign(directions, directions + 3 * n_waves);
        r->solution = (double2 *)solution;
        r->info = info;
        // the path depends on the request alone (and the autotuned table)
        if (r->o.path == 2) {
            bem::TuneEntry te;
            const bool f64 = r->o.precision == BEM_FP64;
            // the autotuned table times the FP32 products: it decides FP32 requests
            const bool mf = !f64 && bem::tune_find(h0->T, std::min(n_waves, 16), &te) &&
                            te.path == 0;
            r->o.path = !mf && bem::dense_bytes(h0, f64) <= srv->o.dense_max_bytes ? 1 : 0;
        }
        BEM_HIP(hipGetDevice(&prev));
        BEM_HIP(hipSetDevice(srv->device));
        r->footprint = bem::solve_footprint(h0, r->k0, r->k1, rho, r->o, n_waves);
        // triangle pairs (assembly or matrix-free products) and, on the
        // assembled path, the operator entries each wave's iterations read
        r->work = (double)h0->T * (double)h0->T *
                  (r->o.path != 0 ? 1.0 : std::min(n_waves, 16) * 50.0) +
                  (r->o.path == 1 ? 4.0 * (double)h0->N * (double)h0->N * n_waves * 50.0 / 64.0
                                  : 0.0);
        (void)hipSetDevice(prev);
        prev = -1;
        {
            std::lock_guard<std::mutex> g(srv->mu);
            if (srv->stop) fail(BEM_E_INVAL, "server is shutting down");
            r->id = srv->next_id++;
            r->t_submit = srv->now();
            srv->reqs[r->id] = r;
            srv->queue.push_back(r);
            *request_id = r->id;
        }
        srv->cv_work.notify_all();
        return BEM_OK;
    } catch (const bem::Error &e) {
        if (prev >= 0) (void)hipSetDevice(prev);
        bem::set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        if (prev >= 0) (void)hipSetDevice(prev);
        bem::set_last_error("host allocation failed");
        return BEM_E_NOMEM;
    }
}

}   // namespace

int bem_server_submit(bem_server *srv, int mesh_id, bem_c64 k_ext, bem_c64 k_int, double rho,
                      const double *directions, int n_waves, double tol,
                      const bem_solve_opts *opts, bem_c64 *solution, bem_solve_info *info,
                      int64_t *request_id) {
    return server_submit(srv, mesh_id, k_ext, k_int, rho, nullptr, nullptr, directions, n_waves,
                         tol, opts, solution, info, request_id);
}

int bem_server_submit_multi(bem_server *srv, int mesh_id, bem_c64 k_ext, const bem_c64 *k_int,
                            const double *rho, const double *directions, int n_waves, double tol,
                            const bem_solve_opts *opts, bem_c64 *solution, bem_solve_info *info,
                            int64_t *request_id) {
    if (!k_int || !rho) {
        bem::set_last_error("k_int and rho must not be NULL");
        return BEM_E_INVAL;
    }
    return server_submit(srv, mesh_id, k_ext, k_int[0], rho[0], k_int, rho, directions, n_waves,
                         tol, opts, solution, info, request_id);
}

int bem_server_wait(bem_server *srv, int64_t request_id, double timeout_s,
                    bem_request_stats *stats) {
    if (!srv) {
        bem::set_last_error("server is NULL");
        return BEM_E_INVAL;
    }
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(request_id);
    if (it == srv->reqs.end()) {
        bem::set_last_error("unknown request id " + std::to_string(request_id));
        return BEM_E_INVAL;
    }
    std::shared_ptr<bem::Request> r = it->second;
    auto done = [&] { return r->done; };
    if (timeout_s < 0) srv->cv_done.wait(lk, done);
    else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done))
        return BEM_W_PENDING;
    if (stats) {
        stats->status = r->status;
        stats->path = r->o.path;   // 0, 1 or 3 (auto resolved at submission)
        stats->t_submit = r->t_submit;
        stats->t_admit = r->t_admit;
        stats->t_end = r->t_end;
        stats->footprint = r->reserved > 0 ? r->reserved : r->footprint;
        stats->replica = r->replica;
    }
    if (r->status < 0) bem::set_last_error(r->msg);
    srv->reqs.erase(it);
    return BEM_OK;
}

int bem_server_stats_get(bem_server *srv, bem_server_stats *st) {
    if (!srv || !st) {
        bem::set_last_error("server or stats is NULL");
        return BEM_E_INVAL;
    }
    std::lock_guard<std::mutex> g(srv->mu);
    st->budget = srv->o.hbm_budget;
    st->resident_bytes = srv->resident();
    st->reserved_bytes = srv->reserved;
    st->peak_bytes = srv->peak;
    st->inflight = srv->inflight;
    st->peak_inflight = srv->peak_inflight;
    st->queued = (int)srv->queue.size();
    st->completed = srv->completed;
    st->rejected = srv->rejected;
    st->evictions = srv->evictions;
    st->krylov_growth_bytes = srv->grown;
    return BEM_OK;
}

}   // extern "C"

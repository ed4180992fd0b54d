// Serving loop: continuous batching of nested-solve requests on one device.
//
// Each registered gauge configuration stays resident (links + clover).  A
// request waits in a FIFO queue until a slot is free and the device memory
// its solve needs fits the budget; then the slot's worker thread runs it on
// the slot's own HIP stream with the slot's own workspace, so admitted
// requests overlap on the device.  Queued requests with the same
// configuration, kappa, c_sw and solver parameters as the head of the queue
// join its solve as further right-hand sides (up to max_batch), so they
// share every launch; a batched right-hand side gives bitwise the result of
// its own solve.  A slot keeps its workspace between requests (no device
// allocation on the hot path once warm); admission (admit_decide in
// wcl_admit.h) keeps every workspace while the budget allows and releases
// idle ones only when a request would not fit.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "wcl_admit.h"
#include "wcl_kernels.h"

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Job {
    uint64_t ticket = 0;
    wcl_request req{};
    wcl_solver_params params{};
    wcl_lattice* lat = nullptr;
    size_t need = 0;       // estimated workspace bytes of the solve
    uint64_t key = 0;      // lattice and solver parameters the workspace is built for
    uint64_t bkey = 0;     // requests with equal bkey can share one solve
    double t_submit = 0, t_admit = 0;
};

// FNV-1a over the lattice handle and every parameter that sizes the workspace
uint64_t job_key(const wcl_lattice* lat, const wcl_solver_params& p) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (v >> (8 * k)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)(uintptr_t)lat);
    const int f[] = {p.precond, p.even_odd, p.ras.block[0], p.ras.block[1], p.ras.block[2], p.ras.block[3],
                     p.ras.s, p.ras.n_ras, p.ras.n_dominv, p.ras.storage, p.ras.kernel, p.ras.block_solver,
                     p.ras.schwarz};
    for (int v : f) mix((uint64_t)(uint32_t)v);
    return h | 1;   // never 0
}

uint64_t dbits(double v) {
    uint64_t b;
    std::memcpy(&b, &v, sizeof b);
    return b;
}

// FNV-1a over everything that defines the operator and the solve: requests
// with the same value solve the same system up to their sources
uint64_t batch_key(const wcl_lattice* lat, const wcl_request& r, const wcl_solver_params& p) {
    uint64_t h = job_key(lat, p);
    auto mix = [&](uint64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (v >> (8 * k)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix(dbits(r.kappa));
    mix(dbits(r.csw));
    mix(dbits(p.tol_outer));
    mix(dbits(p.tol_inner));
    const int f[] = {p.max_outer, p.max_inner, p.max_restarts, p.timers, p.ras.arith};
    for (int v : f) mix((uint64_t)(uint32_t)v);
    return h | 1;
}

// the exact test behind an equal batch key: same lattice, couplings and
// every solver parameter (the key only preselects)
bool same_system(const Job& a, const Job& b) {
    const wcl_solver_params &p = a.params, &q = b.params;
    bool same = a.lat == b.lat && a.req.kappa == b.req.kappa && a.req.csw == b.req.csw &&
                p.tol_outer == q.tol_outer && p.tol_inner == q.tol_inner && p.max_outer == q.max_outer &&
                p.max_inner == q.max_inner && p.max_restarts == q.max_restarts && p.precond == q.precond &&
                p.even_odd == q.even_odd && p.timers == q.timers && p.ras.s == q.ras.s &&
                p.ras.n_ras == q.ras.n_ras && p.ras.n_dominv == q.ras.n_dominv && p.ras.storage == q.ras.storage &&
                p.ras.kernel == q.ras.kernel && p.ras.block_solver == q.ras.block_solver &&
                p.ras.schwarz == q.ras.schwarz && p.ras.arith == q.ras.arith;
    for (int mu = 0; mu < 4; ++mu) same = same && p.ras.block[mu] == q.ras.block[mu];
    return same;
}

// workspace key of a solve of nrhs right-hand sides
uint64_t nrhs_key(uint64_t key, int nrhs) { return (key ^ (0x9e3779b97f4a7c15ull * (uint64_t)nrhs)) | 1; }

// default RAS domain: 4 in every direction it divides, else 2, else the extent
int default_block(int L) { return L % 4 == 0 ? 4 : (L % 2 == 0 ? 2 : L); }

}  // namespace

struct wcl_server {
    wcl_ctx* ctx = nullptr;
    uint64_t budget = 0;
    int max_queue = 4096;
    int max_batch = 1;
    std::map<uint64_t, wcl_lattice*> configs;
    std::mutex mu;
    std::condition_variable cv_done;
    std::deque<Job> queue;
    struct Slot {
        std::thread th;
        hipStream_t st = nullptr;
        Workspace* ws = nullptr;
        size_t held = 0;    // bytes the slot's workspace holds
        uint64_t key = 0;   // what that workspace was built for
        bool busy = false;
        std::vector<Job> jobs;   // the requests of the current solve (one rhs each)
        size_t reserved = 0;     // bytes charged at its admission
        std::condition_variable cv;
    };
    std::vector<Slot*> slots;
    std::map<uint64_t, wcl_result> done;
    std::map<uint64_t, bool> known;   // tickets not yet collected
    uint64_t next_ticket = 1;
    size_t reserved = 0;
    bool stop = false;

    size_t resident_bytes() const {
        size_t b = 0;
        for (auto& kv : configs)
            for (int p = 0; p < 3; ++p) b += gauge_bytes(p, kv.second->V) + clover_bytes(p, kv.second->V);
        return b;
    }
    size_t held_bytes() const {
        size_t b = 0;
        for (auto* s : slots) b += s->held;
        return b;
    }

    void release_workspace(Slot* s) {
        wcl_workspace_delete(s->ws);
        s->ws = wcl_workspace_new(ctx);
        s->held = 0;
        s->key = 0;
    }

    // device bytes of one solve of n requests like j (workspace, sources,
    // solutions and the host staging buffer)
    static size_t batch_need(const Job& j, int n) {
        return nested_workspace_bytes(j.lat, &j.params, n) + 2 * spinor_rhs_bytes(WCL_F64, j.lat->V) * n +
               (size_t)j.lat->V * 24 * sizeof(double);
    }

    // Admits queued requests in FIFO order while a slot is free and the
    // budget allows (admit_decide).  The head of the queue takes along the
    // queued requests with its batch key, up to max_batch, when that batch
    // fits; otherwise it goes alone.  Called with mu held.
    void admit() {
        while (!queue.empty()) {
            std::vector<AdmitSlot> st;
            for (auto* s : slots) st.push_back(AdmitSlot{s->busy, s->held, s->key});
            const Job& head = queue.front();
            std::vector<size_t> pick = {0};
            for (size_t q = 1; q < queue.size() && (int)pick.size() < max_batch; ++q)
                if (queue[q].bkey == head.bkey && same_system(queue[q], head)) pick.push_back(q);
            AdmitDecision d{};
            d.slot = -1;
            while (!pick.empty()) {
                const int n = (int)pick.size();
                d = admit_decide(st, budget, resident_bytes(), reserved, n == 1 ? head.need : batch_need(head, n),
                                 n == 1 ? head.key : nrhs_key(head.key, n));
                if (d.slot >= 0 || n == 1) break;
                pick.resize(1);   // the batch does not fit now: try the head alone
            }
            if (d.slot < 0) return;   // head of line waits for a slot or for memory
            Slot* free_slot = slots[d.slot];
            if (d.release_idle)
                for (auto* s : slots)
                    if (!s->busy && s != free_slot && s->held) release_workspace(s);
            if (d.release_slot) release_workspace(free_slot);
            const int n = (int)pick.size();
            const double t = now_s();
            free_slot->jobs.clear();
            for (size_t q : pick) {
                free_slot->jobs.push_back(queue[q]);
                free_slot->jobs.back().t_admit = t;
            }
            for (size_t k = pick.size(); k-- > 0;) queue.erase(queue.begin() + (ptrdiff_t)pick[k]);
            free_slot->reserved = d.charge;
            reserved += d.charge;
            free_slot->key = n == 1 ? free_slot->jobs[0].key : nrhs_key(free_slot->jobs[0].key, n);
            free_slot->busy = true;
            free_slot->cv.notify_one();
        }
    }

    // One nested solve with the slot's requests as its right-hand sides.
    void run_job(Slot* s) {
        const std::vector<Job>& js = s->jobs;
        const Job& j = js[0];
        const int n = (int)js.size();
        wcl_solve_stats stats{};
        std::vector<double> resid(n, -1.0);
        int rc = WCL_OK;
        const int64_t V = j.lat->V;
        const size_t b64 = spinor_rhs_bytes(WCL_F64, V), stage_b = (size_t)V * 24 * sizeof(double);
        void *eta = nullptr, *phi = nullptr, *stage = nullptr;
        workspace_get(s->ws, "srv.eta", b64 * n, &eta, &rc);
        if (rc == WCL_OK) workspace_get(s->ws, "srv.phi", b64 * n, &phi, &rc);
        if (rc == WCL_OK) workspace_get(s->ws, "srv.stage", stage_b, &stage, &rc);
        // the host sources go through one staging buffer, one after the other
        // (stream order keeps each copy behind the previous pack)
        for (int k = 0; k < n && rc == WCL_OK; ++k) {
            if (hipMemcpyAsync(stage, js[k].req.eta_host, stage_b, hipMemcpyHostToDevice, s->st) != hipSuccess)
                rc = WCL_EHIP;
            if (rc == WCL_OK)
                rc = launch_pack_spinor(j.lat->g, WCL_F64, 1, (const double*)stage, (char*)eta + k * b64, b64, s->st);
        }
        if (rc == WCL_OK)
            rc = nested_solve(j.lat, s->ws, &j.params, j.req.kappa, j.req.csw, eta, phi, n, &stats, s->st,
                              resid.data());
        if (rc == WCL_OK || rc == WCL_ENOTCONV) {
            int rc2 = WCL_OK;
            for (int k = 0; k < n && rc2 == WCL_OK; ++k) {
                rc2 = launch_unpack_spinor(j.lat->g, WCL_F64, 1, (const char*)phi + k * b64, b64, (double*)stage,
                                           s->st);
                if (rc2 == WCL_OK &&
                    hipMemcpyAsync(js[k].req.phi_host, stage, stage_b, hipMemcpyDeviceToHost, s->st) != hipSuccess)
                    rc2 = WCL_EHIP;
            }
            if (rc2 == WCL_OK && hipStreamSynchronize(s->st) != hipSuccess) rc2 = WCL_EHIP;
            if (rc2 != WCL_OK) rc = rc2;
        }
        const double t_done = now_s();
        std::lock_guard<std::mutex> g(mu);
        for (int k = 0; k < n; ++k) {
            wcl_result res{};
            res.t_submit = js[k].t_submit;
            res.t_admit = js[k].t_admit;
            res.t_done = t_done;
            res.batch = n;
            res.stats = stats;
            if (n > 1) {
                // the batch's counters, this request's own residual and status
                res.stats.true_resid = resid[k];
                res.stats.converged = rc == WCL_OK || (rc == WCL_ENOTCONV && resid[k] >= 0 &&
                                                       resid[k] <= js[k].params.tol_outer);
                res.status = rc == WCL_ENOTCONV && res.stats.converged ? WCL_OK : rc;
            } else {
                res.status = rc;
            }
            done[js[k].ticket] = res;
        }
        reserved -= s->reserved;
        s->reserved = 0;
        s->held = workspace_bytes(s->ws);
        s->busy = false;
        cv_done.notify_all();
        admit();
    }

    void worker(Slot* s) {
        (void)hipSetDevice(ctx->device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            s->cv.wait(lk, [&] { return s->busy || stop; });
            if (!s->busy && stop) return;
            lk.unlock();
            run_job(s);
            lk.lock();
        }
    }
};

extern "C" {

int wcl_server_create(wcl_ctx* ctx, const wcl_server_params* p, wcl_server** out) {
    if (!ctx || !p || !out || p->max_slots < 1 || p->max_slots > 64 || p->max_queue < 0 || p->max_batch < 0 ||
        p->max_batch > 64) {
        wcl_set_error("wcl_server_create: bad argument");
        return WCL_EINVAL;
    }
    *out = nullptr;
    WCL_HIP(hipSetDevice(ctx->device));
    auto* srv = new wcl_server;
    srv->ctx = ctx;
    srv->budget = p->hbm_budget_bytes ? p->hbm_budget_bytes : ctx->budget;
    srv->max_queue = p->max_queue ? p->max_queue : 4096;
    srv->max_batch = p->max_batch > 1 ? p->max_batch : 1;
    for (int k = 0; k < p->max_slots; ++k) {
        auto* s = new wcl_server::Slot;
        if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            wcl_server_destroy(srv);
            wcl_set_error("wcl_server_create: stream creation failed");
            return WCL_EHIP;
        }
        s->ws = wcl_workspace_new(ctx);
        srv->slots.push_back(s);
    }
    for (auto* s : srv->slots) s->th = std::thread([srv, s] { srv->worker(s); });
    *out = srv;
    return WCL_OK;
}

int wcl_server_destroy(wcl_server* srv) {
    if (!srv) return WCL_OK;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->cv_done.wait(lk, [&] {
            if (!srv->queue.empty()) return false;
            for (auto* s : srv->slots)
                if (s->busy) return false;
            return true;
        });
        srv->stop = true;
        for (auto* s : srv->slots) s->cv.notify_one();
    }
    for (auto* s : srv->slots) {
        if (s->th.joinable()) s->th.join();
        wcl_workspace_delete(s->ws);
        if (s->st) (void)hipStreamDestroy(s->st);
        delete s;
    }
    for (auto& kv : srv->configs) wcl_destroy_lattice(kv.second);
    delete srv;
    return WCL_OK;
}

int wcl_register_gauge(wcl_server* srv, uint64_t config_id, const int dims[4], const double* U_host) {
    if (!srv || !dims || !U_host) {
        wcl_set_error("wcl_register_gauge: null argument");
        return WCL_EINVAL;
    }
    {
        std::lock_guard<std::mutex> g(srv->mu);
        if (srv->configs.count(config_id)) {
            wcl_set_error("wcl_register_gauge: config %llu already registered", (unsigned long long)config_id);
            return WCL_EINVAL;
        }
        int64_t V = 1;
        for (int mu = 0; mu < 4; ++mu) V *= dims[mu] > 0 ? dims[mu] : 1;
        size_t fields = 0;
        for (int p = 0; p < 3; ++p) fields += gauge_bytes(p, V) + clover_bytes(p, V);
        if (srv->resident_bytes() + srv->held_bytes() + srv->reserved + fields > srv->budget) {
            wcl_set_error("wcl_register_gauge: resident fields (%llu bytes) exceed the server budget",
                          (unsigned long long)fields);
            return WCL_ENOMEM;
        }
    }
    wcl_lattice* lat = nullptr;
    WCL_CHECK(wcl_create_lattice(srv->ctx, dims, nullptr, &lat));
    int rc = wcl_upload_gauge(lat, U_host);
    if (rc == WCL_OK) rc = wcl_compute_clover(lat);
    if (rc != WCL_OK) {
        wcl_destroy_lattice(lat);
        return rc;
    }
    std::lock_guard<std::mutex> g(srv->mu);
    srv->configs[config_id] = lat;
    return WCL_OK;
}

int wcl_submit(wcl_server* srv, const wcl_request* req, uint64_t* ticket) {
    if (!srv || !req || !ticket || !req->eta_host || !req->phi_host) {
        wcl_set_error("wcl_submit: null argument");
        return WCL_EINVAL;
    }
    std::lock_guard<std::mutex> g(srv->mu);
    auto it = srv->configs.find(req->config_id);
    if (it == srv->configs.end()) {
        wcl_set_error("wcl_submit: unknown config %llu", (unsigned long long)req->config_id);
        return WCL_EINVAL;
    }
    Job j;
    j.req = *req;
    j.lat = it->second;
    if (req->params) {
        j.params = *req->params;
    } else {
        j.params.tol_outer = 1e-10;
        j.params.tol_inner = 1e-4;
        j.params.max_outer = 100;
        j.params.max_inner = 100;
        j.params.max_restarts = 10;
        j.params.precond = WCL_PRECOND_RAS;
        for (int mu = 0; mu < 4; ++mu) j.params.ras.block[mu] = default_block(j.lat->g.L[mu]);
        j.params.ras.s = 0;
        j.params.ras.n_ras = 3;
        j.params.ras.n_dominv = 4;
        j.params.ras.storage = WCL_F16;
        j.params.ras.kernel = WCL_BLOCK_AUTO;
    }
    if (j.params.precond == WCL_PRECOND_RAS) {
        Blocks B;
        WCL_CHECK(make_blocks(j.lat, &j.params.ras, &B));
    }
    j.need = nested_workspace_bytes(j.lat, &j.params, 1) + 2 * spinor_rhs_bytes(WCL_F64, j.lat->V) +
             (size_t)j.lat->V * 24 * sizeof(double);
    j.key = job_key(j.lat, j.params);
    j.bkey = batch_key(j.lat, j.req, j.params);
    if (srv->resident_bytes() + j.need > srv->budget) {
        wcl_set_error("wcl_submit: request needs %llu bytes, more than the budget leaves",
                      (unsigned long long)j.need);
        return WCL_ENOMEM;
    }
    if ((int)srv->queue.size() >= srv->max_queue) {
        wcl_set_error("wcl_submit: queue full");
        return WCL_ENOMEM;
    }
    j.ticket = srv->next_ticket++;
    j.t_submit = now_s();
    srv->known[j.ticket] = true;
    srv->queue.push_back(j);
    *ticket = j.ticket;
    srv->admit();
    return WCL_OK;
}

int wcl_poll(wcl_server* srv, uint64_t ticket, wcl_result* res) {
    if (!srv || !res) return WCL_EINVAL;
    std::lock_guard<std::mutex> g(srv->mu);
    if (!srv->known.count(ticket)) {
        wcl_set_error("wcl_poll: unknown ticket %llu", (unsigned long long)ticket);
        return WCL_EINVAL;
    }
    auto it = srv->done.find(ticket);
    if (it == srv->done.end()) return WCL_PENDING;
    *res = it->second;
    srv->done.erase(it);
    srv->known.erase(ticket);
    return WCL_OK;
}

int wcl_wait(wcl_server* srv, uint64_t ticket, wcl_result* res) {
    if (!srv || !res) return WCL_EINVAL;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        if (!srv->known.count(ticket)) {
            wcl_set_error("wcl_wait: unknown ticket %llu", (unsigned long long)ticket);
            return WCL_EINVAL;
        }
        srv->cv_done.wait(lk, [&] { return srv->done.count(ticket) > 0; });
    }
    return wcl_poll(srv, ticket, res);
}

}  // extern "C"

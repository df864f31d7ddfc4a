// serve.cpp -- the solve server behind tmq_server_* (contract in include/tmq.h).
//
// One worker thread drives every CG engine without blocking on any of them:
// per pass it finishes the steps whose scalars have reached the host, takes
// the finished slots (their solutions are copied out on the engine's stream
// and a completion event is recorded behind the copy), joins queued requests
// into free slots, and begins the next step.  Each engine has its own stream,
// so engines of different lattice sizes overlap on the device; the host never
// waits for one engine while another could be fed.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.h"
#include "lattice.h"

namespace tmq {
namespace {

using Clock = std::chrono::steady_clock;

double since(Clock::time_point t0, Clock::time_point t) { return std::chrono::duration<double>(t - t0).count(); }

enum ReqState { Q_WAIT = 0, Q_RUN = 1, Q_COPY = 2, Q_DONE = 3 };

struct EngineRec;

struct Request {
    uint64_t ticket = 0;
    int lat = 0;
    tmq_params p{};
    tmq_solver_opts o{};
    const double2 *b = nullptr;
    double2 *x = nullptr;
    size_t slot_bytes = 0;
    int state = Q_WAIT;
    EngineRec *eng = nullptr;
    int slot = -1;
    hipEvent_t done_ev = nullptr;
    tmq_solve_info info{};
    Clock::time_point t_submit, t_admit, t_done;
};

struct EngineRec {
    std::unique_ptr<Engine> E;
    hipStream_t st = nullptr;
    int lat = 0, sloppy = 0, link_fmt = 0, mode = 0;
    double theta[4] = {0, 0, 0, 0};
    std::vector<Request *> slot_req;  // request in each slot (nullptr: free)
    bool broken = false;
};

struct LatRec {
    std::unique_ptr<Lattice> L;
};

}  // namespace

struct Server {
    int device = 0;
    size_t budget = 0;
    int max_batch = 16;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    bool failed = false;
    std::string fail_msg;
    uint64_t next_ticket = 1;
    std::deque<Request *> queue;                          // waiting for admission (worker and submit)
    std::unordered_map<uint64_t, Request *> by_ticket;    // every unretired request
    std::vector<std::unique_ptr<LatRec>> lats;            // append-only

    // worker-owned
    std::vector<std::unique_ptr<EngineRec>> engines;
    std::vector<Request *> copying;  // solutions being copied out
    std::vector<hipEvent_t> ev_pool;

    // statistics (under mu)
    int n_engines = 0;  // engines.size(), kept here for the stats readers
    size_t bytes_in_use = 0, peak_bytes = 0;
    int running = 0, peak_running = 0;
    long submitted = 0, completed = 0, failed_n = 0, rejected = 0, steps = 0;
    bool have_first = false;
    Clock::time_point t_first, t_last;
    std::vector<double> lat_s, wait_s;

    std::thread worker;

    void run();
    bool pass();
    void admit(std::vector<Request *> &pending, std::vector<Request *> &failed_join);
    EngineRec *engine_for(Request *r, bool may_create, int *err = nullptr);
    int link_fmt_of(const Request *r);
    bool same_key(const EngineRec *er, const Request *r, int lkf) const;
    void fail_engine(EngineRec *er, const std::string &msg);
    void complete(Request *r, int status);
    hipEvent_t get_event();
};

hipEvent_t Server::get_event()
{
    if (!ev_pool.empty()) {
        hipEvent_t e = ev_pool.back();
        ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// called with mu held
void Server::complete(Request *r, int status)
{
    r->state = Q_DONE;
    r->t_done = Clock::now();
    r->info.status = status;
    r->info.seconds = since(r->t_submit, r->t_done);
    completed++;
    if (status != TMQ_OK) failed_n++;
    lat_s.push_back(r->info.seconds);
    wait_s.push_back(since(r->t_submit, r->t_admit));
    t_last = r->t_done;
    cv_done.notify_all();
}

void Server::fail_engine(EngineRec *er, const std::string &msg)
{
    std::lock_guard<std::mutex> lk(mu);
    er->broken = true;
    failed = true;
    fail_msg = msg;
    for (auto &r : er->slot_req)
        if (r) {
            complete(r, TMQ_EDEVICE);
            running--;
            r = nullptr;
        }
}

// The inner link format a request's solve uses (its engine key's last part).
int Server::link_fmt_of(const Request *r)
{
    Lattice *L = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu);
        L = lats[r->lat]->L.get();
    }
    const int sp = r->o.sloppy;
    return sp == P64 ? link_fmt_for(L, P64, P64) : link_fmt_for(L, sp, r->o.sloppy_link);
}

// Whether engine er serves requests like r: same lattice, inner spinor
// precision, inner link format and solver mode (theta is checked apart,
// since an empty engine takes on the theta of the request that joins it).
bool Server::same_key(const EngineRec *er, const Request *r, int lkf) const
{
    return er->lat == r->lat && er->sloppy == r->o.sloppy && er->link_fmt == lkf && er->mode == r->o.mode;
}

// An engine with a free slot for r; may create one within the budget,
// releasing idle engines of other keys for it.  Called without mu.
EngineRec *Server::engine_for(Request *r, bool may_create, int *err)
{
    if (err) *err = TMQ_OK;
    Lattice *L = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu);
        L = lats[r->lat]->L.get();
    }
    const int sp = r->o.sloppy;
    const int lkf = link_fmt_of(r);
    for (auto &er : engines) {
        if (er->broken || !same_key(er.get(), r, lkf) || er->E->body_pending) continue;
        if (engine_free_slot(er->E.get()) < 0) continue;
        const bool empty = engine_occupied(er->E.get()) == 0;
        if (!empty && memcmp(er->theta, r->p.theta, sizeof(er->theta)) != 0) continue;
        return er.get();
    }
    if (!may_create) return nullptr;
    // a new engine: as many slots as the budget allows, up to max_batch
    const size_t one = engine_bytes(L, sp, 1, r->o.mode);
    size_t in_use;
    {
        std::lock_guard<std::mutex> lk(mu);
        in_use = bytes_in_use;
    }
    if (in_use + one > budget) {
        // release idle engines (no occupied slot, nothing in flight) of other keys
        for (size_t i = 0; i < engines.size();) {
            EngineRec *er = engines[i].get();
            if (engine_occupied(er->E.get()) == 0 && !er->E->body_pending && !same_key(er, r, lkf)) {
                bool copying_from = false;
                for (Request *q : copying) copying_from |= q->eng == er;
                if (!copying_from) {
                    const size_t b = er->E->bytes;
                    er->E.reset();
                    hipStreamDestroy(er->st);
                    std::lock_guard<std::mutex> lk(mu);
                    engines.erase(engines.begin() + (long)i);
                    n_engines = (int)engines.size();
                    bytes_in_use -= b;
                    in_use = bytes_in_use;
                    continue;
                }
            }
            i++;
        }
        if (in_use + one > budget) return nullptr;
    }
    int cap = max_batch;
    while (cap > 1 && in_use + engine_bytes(L, sp, cap, r->o.mode) > budget) cap--;
    auto er = std::make_unique<EngineRec>();
    if (hipStreamCreateWithFlags(&er->st, hipStreamNonBlocking) != hipSuccess) {
        if (err) *err = TMQ_EDEVICE;
        return nullptr;
    }
    Engine *E = nullptr;
    const int cs = engine_create(L, sp, r->o.sloppy_link, r->o.mode, cap, er->st, &E);
    if (cs != TMQ_OK) {
        hipStreamDestroy(er->st);
        if (err) *err = cs;
        return nullptr;
    }
    er->E.reset(E);
    er->lat = r->lat;
    er->sloppy = sp;
    er->link_fmt = lkf;
    er->mode = r->o.mode;
    memcpy(er->theta, r->p.theta, sizeof(er->theta));
    er->slot_req.assign(cap, nullptr);
    std::lock_guard<std::mutex> lk(mu);
    bytes_in_use += E->bytes;
    peak_bytes = std::max(peak_bytes, bytes_in_use);
    engines.push_back(std::move(er));
    n_engines = (int)engines.size();
    return engines.back().get();
}

// Join waiting requests in arrival order.  A request whose engine has no
// free slot waits for one while later requests of other keys go ahead.  A
// request that has no engine and no memory for one blocks every later
// request: the engines then drain, become idle and are released for it, so
// no lattice size can be starved by a stream of others.
void Server::admit(std::vector<Request *> &pending, std::vector<Request *> &failed_join)
{
    std::vector<Request *> still;
    bool blocked = false;
    for (Request *r : pending) {
        EngineRec *er = blocked ? nullptr : engine_for(r, false);
        if (!er && !blocked) {
            // an engine of the request's own key (the key engine_for matches on)
            // that will free a slot: wait for it; otherwise create one
            const int lkf = link_fmt_of(r);
            bool has_engine = false;
            for (auto &e : engines)
                has_engine |= !e->broken && same_key(e.get(), r, lkf) &&
                              memcmp(e->theta, r->p.theta, sizeof(e->theta)) == 0;
            if (!has_engine) {
                int err = TMQ_OK;
                er = engine_for(r, true, &err);
                if (!er && err != TMQ_OK && engines.empty()) {
                    // the device refused memory that the budget allowed, and no
                    // engine will ever release any: fail rather than wait
                    r->t_admit = Clock::now();
                    r->info.status = err;
                    failed_join.push_back(r);
                    continue;
                }
                if (!er) blocked = true;
            }
        }
        if (!er) {
            still.push_back(r);
            continue;
        }
        Engine *E = er->E.get();
        const int slot = engine_free_slot(E);
        r->t_admit = Clock::now();
        if (engine_occupied(E) == 0) memcpy(er->theta, r->p.theta, sizeof(er->theta));
        if (engine_join(E, slot, r->p, r->o, r->b) != TMQ_OK) {
            fail_engine(er, get_error());
            failed_join.push_back(r);  // completed once it has left the queue
            continue;
        }
        er->slot_req[slot] = r;
        r->eng = er;
        r->slot = slot;
        std::lock_guard<std::mutex> lk(mu);
        r->state = Q_RUN;
        running++;
        peak_running = std::max(peak_running, running);
    }
    pending.swap(still);
}

// one pass over everything; true if anything progressed
bool Server::pass()
{
    bool progress = false;
    // finished copies
    for (size_t i = 0; i < copying.size();) {
        Request *r = copying[i];
        const hipError_t q = hipEventQuery(r->done_ev);
        if (q == hipErrorNotReady) {
            i++;
            continue;
        }
        ev_pool.push_back(r->done_ev);
        r->done_ev = nullptr;
        {
            std::lock_guard<std::mutex> lk(mu);
            complete(r, q == hipSuccess ? r->info.status : TMQ_EDEVICE);
        }
        copying.erase(copying.begin() + (long)i);
        progress = true;
    }
    // steps that can be finished
    for (auto &erp : engines) {
        EngineRec *er = erp.get();
        Engine *E = er->E.get();
        if (er->broken || !E->body_pending || !engine_ready(E)) continue;
        std::vector<int> fin;
        if (engine_end_step(E, &fin) != TMQ_OK) {
            fail_engine(er, get_error());
            continue;
        }
        progress = true;
        {
            std::lock_guard<std::mutex> lk(mu);
            steps++;
        }
        for (int s : fin) {
            Request *r = er->slot_req[s];
            er->slot_req[s] = nullptr;
            tmq_solve_info info{};
            const int st = engine_take(E, s, r->x, &info);
            r->info = info;
            r->done_ev = get_event();
            {
                std::lock_guard<std::mutex> lk(mu);
                running--;
                r->state = Q_COPY;
            }
            if (st != TMQ_OK || !r->done_ev || hipEventRecord(r->done_ev, er->st) != hipSuccess) {
                if (r->done_ev) ev_pool.push_back(r->done_ev);
                r->done_ev = nullptr;
                std::lock_guard<std::mutex> lk(mu);
                complete(r, TMQ_EDEVICE);
                continue;
            }
            copying.push_back(r);
        }
    }
    // admissions
    std::vector<Request *> pending, failed_join;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!stop) pending.assign(queue.begin(), queue.end());
    }
    if (!pending.empty()) {
        const size_t before = pending.size();
        admit(pending, failed_join);
        if (pending.size() != before) {
            progress = true;
            std::lock_guard<std::mutex> lk(mu);
            // keep the still-waiting ones (and whatever arrived meanwhile) in order
            std::deque<Request *> q;
            for (Request *r : queue)
                if (r->state == Q_WAIT && std::find(failed_join.begin(), failed_join.end(), r) == failed_join.end())
                    q.push_back(r);
            queue.swap(q);
            for (Request *r : failed_join) {
                r->t_admit = Clock::now();
                complete(r, r->info.status == TMQ_ENOMEM ? TMQ_ENOMEM : TMQ_EDEVICE);
            }
        }
    }
    // begin the next step of engines with work
    for (auto &erp : engines) {
        EngineRec *er = erp.get();
        Engine *E = er->E.get();
        if (er->broken || E->body_pending || engine_running(E) == 0) continue;
        if (engine_begin_step(E) != TMQ_OK) {
            fail_engine(er, get_error());
            continue;
        }
        progress = true;
    }
    return progress;
}

void Server::run()
{
    hipSetDevice(device);
    for (;;) {
        const bool progress = pass();
        std::unique_lock<std::mutex> lk(mu);
        const bool in_flight = running > 0 || !copying.empty();
        if (stop && !in_flight) break;
        if (progress) continue;
        if (in_flight) {
            // the device is busy: look again at once (a step of a small
            // lattice lasts tens of microseconds)
            lk.unlock();
            std::this_thread::yield();
        } else if (!queue.empty() && !stop) {
            // waiting for memory that only a finishing request can free
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        } else {
            cv_work.wait_for(lk, std::chrono::milliseconds(50));
        }
    }
    // drop the requests still queued
    std::lock_guard<std::mutex> lk(mu);
    queue.clear();
}

}  // namespace tmq

struct tmq_server {
    tmq::Server S;
};

using namespace tmq;

namespace {

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev)
    {
        hipGetDevice(&prev);
        hipSetDevice(dev);
    }
    ~DevGuard()
    {
        if (prev >= 0) hipSetDevice(prev);
    }
};

int retire(Server &S, Request *r, tmq_solve_info *info)
{
    const int st = r->info.status;
    if (info) *info = r->info;
    S.by_ticket.erase(r->ticket);
    delete r;
    return st;
}

}  // namespace

extern "C" {

int tmq_server_create(int device, const tmq_server_config *cfg, tmq_server **out)
{
    if (!out) {
        set_error("tmq_server_create: NULL out");
        return TMQ_EINVAL;
    }
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        set_error("tmq_server_create: no such HIP device");
        return TMQ_EDEVICE;
    }
    if (cfg && cfg->max_batch > TMQ_MAX_RHS) {
        set_error("tmq_server_create: max_batch above TMQ_MAX_RHS");
        return TMQ_EINVAL;
    }
    DevGuard dg(device);
    size_t budget = cfg ? cfg->budget_bytes : 0;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            set_error("tmq_server_create: hipMemGetInfo failed");
            return TMQ_EDEVICE;
        }
        budget = (size_t)(0.6 * (double)fr);
    }
    tmq_server *srv = new tmq_server();
    Server &S = srv->S;
    S.device = device;
    S.budget = budget;
    S.max_batch = cfg && cfg->max_batch > 0 ? cfg->max_batch : 16;
    S.worker = std::thread([&S] { S.run(); });
    *out = srv;
    return TMQ_OK;
}

int tmq_server_add_lattice(tmq_server *srv, const int dims[4], const double *U_dev, int *lattice_id)
{
    if (!srv || !dims || !U_dev || !lattice_id) {
        set_error("tmq_server_add_lattice: NULL argument");
        return TMQ_EINVAL;
    }
    Server &S = srv->S;
    DevGuard dg(S.device);
    Lattice *L = nullptr;
    TMQ_TRY(lattice_create(dims, S.device, &L));
    std::unique_ptr<Lattice> hold(L);
    TMQ_TRY(lattice_load_gauge(L, (const double2 *)U_dev, L->own));
    std::lock_guard<std::mutex> lk(S.mu);
    auto rec = std::make_unique<LatRec>();
    rec->L = std::move(hold);
    S.lats.push_back(std::move(rec));
    *lattice_id = (int)S.lats.size() - 1;
    return TMQ_OK;
}

int tmq_server_submit(tmq_server *srv, int lattice_id, const tmq_params *p, const tmq_solver_opts *opts,
                      const double *b_dev, double *x_dev, uint64_t *ticket)
{
    if (!srv || !ticket || !b_dev || !x_dev) {
        set_error("tmq_server_submit: NULL argument");
        return TMQ_EINVAL;
    }
    TMQ_TRY(check_params(p));
    TMQ_TRY(check_opts(opts));
    if (opts->mode == TMQ_MODE_BICGSTAB) {
        set_error("tmq_server_submit: the server solves the normal equations by CG (mode 0 or 1)");
        return TMQ_EINVAL;
    }
    Server &S = srv->S;
    std::unique_lock<std::mutex> lk(S.mu);
    if (S.failed) {
        set_error("tmq_server_submit: the server has failed: " + S.fail_msg);
        return TMQ_EDEVICE;
    }
    if (lattice_id < 0 || lattice_id >= (int)S.lats.size()) {
        set_error("tmq_server_submit: unknown lattice id");
        return TMQ_EINVAL;
    }
    const Lattice *L = S.lats[lattice_id]->L.get();
    const size_t one = engine_bytes(L, opts->sloppy, 1, opts->mode);
    if (one > S.budget) {
        S.rejected++;
        set_error("tmq_server_submit: one solve on this lattice needs more device memory than the budget");
        return TMQ_ENOMEM;
    }
    Request *r = new Request();
    r->ticket = S.next_ticket++;
    r->lat = lattice_id;
    r->p = *p;
    r->o = *opts;
    r->b = (const double2 *)b_dev;
    r->x = (double2 *)x_dev;
    r->slot_bytes = one;
    r->t_submit = Clock::now();
    if (!S.have_first) {
        S.have_first = true;
        S.t_first = r->t_submit;
    }
    S.submitted++;
    S.queue.push_back(r);
    S.by_ticket[r->ticket] = r;
    *ticket = r->ticket;
    lk.unlock();
    S.cv_work.notify_one();
    return TMQ_OK;
}

int tmq_server_poll(tmq_server *srv, uint64_t ticket, tmq_solve_info *info)
{
    if (!srv) {
        set_error("tmq_server_poll: NULL server");
        return TMQ_EINVAL;
    }
    Server &S = srv->S;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.by_ticket.find(ticket);
    if (it == S.by_ticket.end()) {
        set_error("tmq_server_poll: unknown or retired ticket");
        return TMQ_EINVAL;
    }
    if (it->second->state != Q_DONE) return TMQ_PENDING;
    return retire(S, it->second, info);
}

int tmq_server_wait(tmq_server *srv, uint64_t ticket, double timeout_s, tmq_solve_info *info)
{
    if (!srv) {
        set_error("tmq_server_wait: NULL server");
        return TMQ_EINVAL;
    }
    Server &S = srv->S;
    std::unique_lock<std::mutex> lk(S.mu);
    const auto deadline = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                             std::chrono::duration<double>(timeout_s < 0 ? 0.0 : timeout_s));
    for (;;) {
        auto it = S.by_ticket.find(ticket);
        if (it == S.by_ticket.end()) {
            set_error("tmq_server_wait: unknown or retired ticket");
            return TMQ_EINVAL;
        }
        if (it->second->state == Q_DONE) return retire(S, it->second, info);
        if (timeout_s >= 0 && Clock::now() >= deadline) return TMQ_PENDING;
        if (timeout_s < 0)
            S.cv_done.wait_for(lk, std::chrono::milliseconds(100));
        else
            S.cv_done.wait_until(lk, deadline);
    }
}

static double percentile(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

int tmq_server_get_stats(tmq_server *srv, tmq_server_stats *out)
{
    if (!srv || !out) {
        set_error("tmq_server_get_stats: NULL argument");
        return TMQ_EINVAL;
    }
    Server &S = srv->S;
    std::lock_guard<std::mutex> lk(S.mu);
    tmq_server_stats o{};
    o.submitted = S.submitted;
    o.completed = S.completed;
    o.failed = S.failed_n;
    o.rejected = S.rejected;
    o.queued = (long)S.queue.size();
    o.running = S.running;
    o.p50_s = percentile(S.lat_s, 0.50);
    o.p99_s = percentile(S.lat_s, 0.99);
    double m = 0.0, w = 0.0;
    for (double v : S.lat_s) m += v;
    for (double v : S.wait_s) w += v;
    o.mean_s = S.lat_s.empty() ? 0.0 : m / (double)S.lat_s.size();
    o.mean_wait_s = S.wait_s.empty() ? 0.0 : w / (double)S.wait_s.size();
    o.elapsed_s = S.have_first && S.completed ? since(S.t_first, S.t_last) : 0.0;
    o.solves_per_s = o.elapsed_s > 0 ? (double)S.completed / o.elapsed_s : 0.0;
    o.budget_bytes = S.budget;
    o.bytes_in_use = S.bytes_in_use;
    o.peak_bytes = S.peak_bytes;
    o.engines = S.n_engines;
    o.peak_running = S.peak_running;
    o.steps = S.steps;
    *out = o;
    return TMQ_OK;
}

int tmq_server_reset_stats(tmq_server *srv)
{
    if (!srv) {
        set_error("tmq_server_reset_stats: NULL server");
        return TMQ_EINVAL;
    }
    Server &S = srv->S;
    std::lock_guard<std::mutex> lk(S.mu);
    S.submitted = S.completed = S.failed_n = S.rejected = S.steps = 0;
    S.have_first = false;
    S.lat_s.clear();
    S.wait_s.clear();
    S.peak_bytes = S.bytes_in_use;
    S.peak_running = S.running;
    return TMQ_OK;
}

void tmq_server_destroy(tmq_server *srv)
{
    if (!srv) return;
    Server &S = srv->S;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.stop = true;
    }
    S.cv_work.notify_all();
    if (S.worker.joinable()) S.worker.join();
    DevGuard dg(S.device);
    for (auto &er : S.engines) {
        er->E.reset();
        if (er->st) hipStreamDestroy(er->st);
    }
    S.engines.clear();
    for (hipEvent_t e : S.ev_pool) hipEventDestroy(e);
    for (auto &kv : S.by_ticket) delete kv.second;
    S.by_ticket.clear();
    S.lats.clear();
    delete srv;
}

}  // extern "C"

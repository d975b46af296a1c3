// Serving loop: ground-state solves of many TPB problems on one device with
// continuous batching.
//
//   submit   validates and deep-copies a request, rejects one whose device
//            footprint exceeds the whole budget, and queues it (FCFS);
//   prep     (one thread) admits queued requests in arrival order while
//            their footprint bound fits the HBM budget, later requests
//            filling in when the head does not fit; builds the context and
//            the solver state on its own stream, trims the reservation to
//            the bytes actually held, and frees finished requests;
//   engine   (one thread) runs the batched Davidson over every admitted
//            request of at most batch_ndet_threshold determinants: new
//            requests join between rounds, so small problems share their
//            sigma and vector launches, and their subspaces stay in HBM for
//            the whole solve;
//   solo     (two threads) solve larger requests with the single-problem
//            solver, each on its own stream, overlapping the engine.
//
// A failed request (bad input at submit, device allocation failure while
// building) ends with an error status of its own; the others go on.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "batch.hpp"

namespace tbsci {
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    int M = 0, na = 0, nb = 0;
    std::vector<double> h, eri;
    std::vector<uint64_t> a, b;
    tbsci_davidson_opts o{};
    int64_t n_det = 0;
    bool batched = false;
    size_t reserved = 0;   // bytes counted against the budget while it runs
    size_t footprint = 0;  // device bytes the request held (its bound until built)
    enum { kQueued, kRunning, kDone } state = kQueued;
    int status = TBSCI_PENDING;
    std::string msg;
    tbsci_davidson_info info{};
    Clock::time_point t_submit, t_start, t_done;
    Ctx *ctx = nullptr;
    BatchSlot *slot = nullptr;
};

size_t request_bound(const Request &r, bool batched) {
    // a batched request with identical lists solves its two spin-flip
    // sectors in two slots at the same time; the solo solver runs them one
    // after the other in one
    const bool two = batched && r.na == r.nb && r.a == r.b && r.a.size() > 1 && r.o.sector == 0;
    const size_t solver = BatchEngine::slot_bytes(r.n_det, r.o) * (two ? 2 : 1);
    return ctx_bytes_bound(r.M, r.na, r.nb, (int64_t)r.a.size(), (int64_t)r.b.size()) + solver;
}

}  // namespace

struct Server {
    int device = 0;
    size_t budget = 0;
    int64_t thresh = 0;
    std::mutex mu;
    std::condition_variable cv_prep, cv_eng, cv_solo;
    std::deque<Request *> queue;
    std::deque<Request *> ready_batch, ready_solo;
    std::vector<Request *> to_free;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_ticket = 1;
    size_t reserved = 0, peak = 0;
    int64_t submitted = 0, completed = 0, failed = 0, running_batched = 0, running_solo = 0;
    int64_t ticks = 0;
    int max_batch = 0;
    std::atomic<bool> stop{false};
    std::thread prep, eng;
    std::vector<std::thread> solo;

    void complete(Request *r, int status, const std::string &msg) {  // with mu held
        r->status = status;
        r->msg = msg;
        r->state = Request::kDone;
        r->t_done = Clock::now();
        ++completed;
        if (status != TBSCI_OK && status != TBSCI_E_NOTCONV) ++failed;
        to_free.push_back(r);
        cv_prep.notify_one();
    }

    // first queued request whose bound fits the free budget (mu held)
    Request *admit() {
        for (auto it = queue.begin(); it != queue.end(); ++it) {
            Request *r = *it;
            if (r->reserved <= budget - reserved) {
                queue.erase(it);
                reserved += r->reserved;
                peak = std::max(peak, reserved);
                r->state = Request::kRunning;
                r->t_start = Clock::now();
                return r;
            }
        }
        return nullptr;
    }

    void free_request(Request *r) {
        if (r->slot) BatchEngine::free_slot(r->slot);
        r->slot = nullptr;
        if (r->ctx) destroy_ctx(r->ctx);
        r->ctx = nullptr;
        std::vector<double>().swap(r->h);
        std::vector<double>().swap(r->eri);
    }

    void prep_loop() {
        (void)hipSetDevice(device);
        for (;;) {
            std::vector<Request *> frees;
            Request *r = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_prep.wait(lk, [&] {
                    if (stop || !to_free.empty()) return true;
                    for (Request *q : queue)
                        if (q->reserved <= budget - reserved) return true;
                    return false;
                });
                frees.swap(to_free);
                if (!stop) r = admit();
            }
            if (!frees.empty()) {
                size_t back = 0;
                for (Request *f : frees) {
                    free_request(f);
                    back += f->reserved;
                }
                std::lock_guard<std::mutex> lk(mu);
                reserved -= back;
                for (Request *f : frees) f->reserved = 0;
            }
            if (!r) {
                if (stop) break;
                continue;
            }
            try {
                r->ctx = create_ctx(r->M, r->na, r->nb, r->h.data(), r->eri.data(), r->a.data(),
                                    (int64_t)r->a.size(), r->b.data(), (int64_t)r->b.size(), device);
                reserve_sigma_workspace(*r->ctx);
                size_t held = ctx_bytes(*r->ctx);
                if (r->batched) {
                    r->slot = BatchEngine::make_slot(r->ctx, r->o, false, true);
                    r->slot->user = r;
                    held += r->slot->bytes;
                } else {
                    held += BatchEngine::slot_bytes(r->n_det, r->o);
                }
                std::lock_guard<std::mutex> lk(mu);
                if (held < r->reserved) {  // keep only what the request holds
                    reserved -= r->reserved - held;
                    r->reserved = held;
                }
                r->footprint = held;
                if (r->batched) {
                    ready_batch.push_back(r);
                    cv_eng.notify_one();
                } else {
                    ready_solo.push_back(r);
                    cv_solo.notify_one();
                }
            } catch (const Error &e) {
                std::lock_guard<std::mutex> lk(mu);
                complete(r, e.code, e.what());
            } catch (const std::exception &e) {
                std::lock_guard<std::mutex> lk(mu);
                complete(r, TBSCI_E_DEVICE, e.what());
            }
        }
    }

    void engine_loop() {
        (void)hipSetDevice(device);
        hipStream_t st = nullptr;
        std::unique_ptr<BatchEngine> e;
        try {
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
                throw Error(TBSCI_E_DEVICE, "stream creation failed");
            e.reset(new BatchEngine(device, st));
        } catch (...) {
            // no engine: batched requests fail as they arrive
            for (;;) {
                std::unique_lock<std::mutex> lk(mu);
                cv_eng.wait(lk, [&] { return stop || !ready_batch.empty(); });
                while (!ready_batch.empty()) {
                    complete(ready_batch.front(), TBSCI_E_DEVICE, "batch engine unavailable");
                    ready_batch.pop_front();
                }
                if (stop) break;
            }
            if (st) (void)hipStreamDestroy(st);
            return;
        }
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_eng.wait(lk, [&] { return stop || !ready_batch.empty() || e->active() > 0; });
                if (stop) break;
                while (!ready_batch.empty() &&
                       e->active() + BatchEngine::slots_of(ready_batch.front()->slot) <=
                           (size_t)kBatchMaxSlots) {
                    e->add(ready_batch.front()->slot);
                    ready_batch.pop_front();
                    ++running_batched;
                }
            }
            std::vector<BatchSlot *> done;
            std::string err;
            int code = TBSCI_OK;
            try {
                e->tick();
                done = e->take_done();
            } catch (const Error &x) {
                code = x.code;
                err = x.what();
            } catch (const std::exception &x) {
                code = TBSCI_E_DEVICE;
                err = x.what();
            }
            std::lock_guard<std::mutex> lk(mu);
            ticks = e->ticks;
            max_batch = std::max(max_batch, e->max_group);
            for (BatchSlot *s : done) {
                Request *r = (Request *)s->user;
                r->info = s->info;
                --running_batched;
                complete(r, s->status, s->status == TBSCI_OK ? "" : "not converged");
            }
            if (code != TBSCI_OK) break;  // device error: the loop below fails the rest
        }
        // stop (or a device error): requests still in the engine end here
        {
            std::lock_guard<std::mutex> lk(mu);
            (void)hipStreamSynchronize(st);
            for (BatchSlot *s : e->take_done()) {
                Request *r = (Request *)s->user;
                r->info = s->info;
                --running_batched;
                complete(r, s->status, "");
            }
            for (BatchSlot *s : e->drain()) {
                --running_batched;
                complete((Request *)s->user, TBSCI_E_STATE, "cancelled");
            }
            while (!ready_batch.empty()) {
                complete(ready_batch.front(), TBSCI_E_STATE, "cancelled");
                ready_batch.pop_front();
            }
        }
        e.reset();
        (void)hipStreamDestroy(st);
    }

    void solo_loop() {
        (void)hipSetDevice(device);
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
        for (;;) {
            Request *r = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_solo.wait(lk, [&] { return stop || !ready_solo.empty(); });
                if (!ready_solo.empty()) {
                    r = ready_solo.front();
                    ready_solo.pop_front();
                    if (stop) {
                        complete(r, TBSCI_E_STATE, "cancelled");
                        continue;
                    }
                    ++running_solo;
                } else if (stop) {
                    break;
                }
            }
            if (!r) continue;
            int rc = TBSCI_OK;
            std::string msg;
            tbsci_davidson_info info{};
            try {
                if (!st) throw Error(TBSCI_E_DEVICE, "stream creation failed");
                rc = solve_one(*r->ctx, r->o, nullptr, nullptr, info, st, &stop);
                if (rc == TBSCI_E_STATE) msg = "cancelled";
            } catch (const Error &x) {
                rc = x.code;
                msg = x.what();
            } catch (const std::exception &x) {
                rc = TBSCI_E_DEVICE;
                msg = x.what();
            }
            std::lock_guard<std::mutex> lk(mu);
            r->info = info;
            --running_solo;
            complete(r, rc, msg);
        }
        if (st) (void)hipStreamDestroy(st);
    }
};

}  // namespace tbsci

using namespace tbsci;

extern "C" {

int tbsci_server_create(int device, size_t hbm_budget_bytes, int64_t batch_ndet_threshold,
                        tbsci_server **out) {
    return guarded([&]() -> int {
        if (!out) throw Error(TBSCI_E_INVAL, "out is NULL");
        if (hbm_budget_bytes == 0) throw Error(TBSCI_E_INVAL, "hbm_budget_bytes must be positive");
        if (batch_ndet_threshold < 0)
            throw Error(TBSCI_E_INVAL, "batch_ndet_threshold must be >= 0");
        check_device_index(device);
        TB_HIP(hipSetDevice(device));
        auto *s = new Server();
        s->device = device;
        s->budget = hbm_budget_bytes;
        s->thresh = batch_ndet_threshold;
        try {
            s->prep = std::thread([s] { s->prep_loop(); });
            s->eng = std::thread([s] { s->engine_loop(); });
            for (int i = 0; i < 2; ++i) s->solo.emplace_back([s] { s->solo_loop(); });
        } catch (...) {
            s->stop = true;
            s->cv_prep.notify_all();
            s->cv_eng.notify_all();
            s->cv_solo.notify_all();
            if (s->prep.joinable()) s->prep.join();
            if (s->eng.joinable()) s->eng.join();
            for (auto &t : s->solo)
                if (t.joinable()) t.join();
            delete s;
            throw Error(TBSCI_E_NOMEM, "could not start the server threads");
        }
        *out = (tbsci_server *)s;
        return TBSCI_OK;
    });
}

void tbsci_server_destroy(tbsci_server *srv) {
    if (!srv) return;
    auto *s = (Server *)srv;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        while (!s->queue.empty()) {
            s->complete(s->queue.front(), TBSCI_E_STATE, "cancelled");
            s->queue.pop_front();
        }
    }
    s->cv_eng.notify_all();
    s->cv_solo.notify_all();
    if (s->eng.joinable()) s->eng.join();
    for (auto &t : s->solo)
        if (t.joinable()) t.join();
    s->cv_prep.notify_all();
    if (s->prep.joinable()) s->prep.join();
    (void)hipSetDevice(s->device);
    for (auto &kv : s->reqs) s->free_request(kv.second.get());
    delete s;
}

int tbsci_submit(tbsci_server *srv, int M, int n_alpha, int n_beta, const double *h,
                 const double *eri, const uint64_t *alpha, int64_t l_alpha, const uint64_t *beta,
                 int64_t l_beta, const tbsci_davidson_opts *opts, uint64_t *ticket) {
    return guarded([&]() -> int {
        if (!srv) throw Error(TBSCI_E_INVAL, "server is NULL");
        if (!ticket) throw Error(TBSCI_E_INVAL, "ticket is NULL");
        auto *s = (Server *)srv;
        validate_problem(M, n_alpha, n_beta, h, eri, alpha, l_alpha, beta, l_beta);
        auto r = std::make_unique<Request>();
        if (opts)
            r->o = *opts;
        else
            tbsci_davidson_default_opts(&r->o);
        check_opts(r->o);
        if (r->o.guess_kind != TBSCI_GUESS_DIAG)
            throw Error(TBSCI_E_INVAL, "served solves take no start vector");
        r->M = M;
        r->na = n_alpha;
        r->nb = n_beta;
        const size_t M2 = (size_t)M * M;
        r->h.assign(h, h + M2);
        r->eri.assign(eri, eri + M2 * M2);
        r->a.assign(alpha, alpha + l_alpha);
        r->b.assign(beta, beta + l_beta);
        r->n_det = l_alpha * l_beta;
        r->batched = r->n_det <= s->thresh;
        r->reserved = request_bound(*r, r->batched);
        r->footprint = r->reserved;
        if (r->reserved > s->budget)
            throw Error(TBSCI_E_NOMEM, "request footprint (" + std::to_string(r->reserved) +
                                           " bytes) exceeds the server's HBM budget");
        r->t_submit = Clock::now();
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) throw Error(TBSCI_E_STATE, "server is stopping");
        r->ticket = s->next_ticket++;
        *ticket = r->ticket;
        s->queue.push_back(r.get());
        s->reqs.emplace(r->ticket, std::move(r));
        ++s->submitted;
        s->cv_prep.notify_one();
        return TBSCI_OK;
    });
}

int tbsci_poll(tbsci_server *srv, uint64_t ticket, tbsci_davidson_info *out) {
    return guarded([&]() -> int {
        if (!srv) throw Error(TBSCI_E_INVAL, "server is NULL");
        auto *s = (Server *)srv;
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) throw Error(TBSCI_E_NOTFOUND, "no such ticket");
        const Request &r = *it->second;
        if (r.state != Request::kDone) return TBSCI_PENDING;
        if (out) *out = r.info;
        if (r.status != TBSCI_OK) set_error(r.status, r.msg);
        return r.status;
    });
}

int tbsci_request_times(tbsci_server *srv, uint64_t ticket, double *queue_s, double *latency_s,
                        int *batched, int64_t *footprint_bytes) {
    return guarded([&]() -> int {
        if (!srv) throw Error(TBSCI_E_INVAL, "server is NULL");
        auto *s = (Server *)srv;
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) throw Error(TBSCI_E_NOTFOUND, "no such ticket");
        const Request &r = *it->second;
        if (r.state != Request::kDone) return TBSCI_PENDING;
        auto sec = [](Clock::duration d) { return std::chrono::duration<double>(d).count(); };
        const bool started = r.t_start.time_since_epoch().count() != 0;
        if (queue_s) *queue_s = sec((started ? r.t_start : r.t_done) - r.t_submit);
        if (latency_s) *latency_s = sec(r.t_done - r.t_submit);
        if (batched) *batched = r.batched ? 1 : 0;
        if (footprint_bytes) *footprint_bytes = (int64_t)r.footprint;
        return TBSCI_OK;
    });
}

int tbsci_server_stats(tbsci_server *srv, tbsci_server_info *out) {
    return guarded([&]() -> int {
        if (!srv || !out) throw Error(TBSCI_E_INVAL, "NULL argument");
        auto *s = (Server *)srv;
        std::lock_guard<std::mutex> lk(s->mu);
        out->hbm_budget = s->budget;
        out->hbm_reserved = s->reserved;
        out->hbm_reserved_peak = s->peak;
        out->submitted = s->submitted;
        out->completed = s->completed;
        out->failed = s->failed;
        out->queued = (int64_t)s->queue.size();
        out->running_batched = s->running_batched;
        out->running_solo = s->running_solo;
        out->ticks = s->ticks;
        out->max_batch = s->max_batch;
        return TBSCI_OK;
    });
}

}  // extern "C"

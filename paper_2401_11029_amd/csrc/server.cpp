// server.cpp -- continuous batching of CFL-reachability requests.
//
// A worker thread owns two Runs: one for small requests (device footprint at
// most 1/64 of the budget) and one for the rest.  Between rounds it retires
// the instances that converged (their matrices are compacted to the user
// non-terminals and handed to the waiting caller) and admits queued
// requests in arrival order, each into its class's run, while the estimated
// footprint of the running instances plus the next one fits the budget and
// a slot is free (a request that does not fit yet lets later ones of the
// other class pass).  Every round is one fused product launch over all
// instances of a run, so a request that arrives while others are on the
// device starts at the next round boundary of its run.  The small run takes
// kSmallPace round batches per batch of the large run: its rounds are short,
// so a small request does not wait a large request's round for each of its
// own.  Each instance's arithmetic is independent of the others (its own
// matrices, rows and new pairs), so its result equals a solo solve.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>

#include "engine.h"

using namespace cflr;

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket = 0;
    const cflr_grammar *g = nullptr;
    const cflr_graph *graph = nullptr;
    double t_submit = 0, t_admit = 0, t_finish = 0;
    bool finished = false;
    bool taken = false;
    cflr_status status = CFLR_OK;
    std::string error;
    std::shared_ptr<Instance> inst;
    uint64_t footprint = 0;
    uint64_t slots = 0;  // (key tile, partner) slots of its matrices (instance_pair_slots)
    int cls = 1;         // 0: small, 1: large
};

constexpr uint64_t kSmallShare = 64;  // small: footprint at most budget / kSmallShare
constexpr uint32_t kSmallPace = 2;    // small-run round batches per large-run batch

}  // namespace

struct cflr_server {
    CtxRef hold;  // first member: released last
    cflr_ctx *ctx = nullptr;
    cflr_opts opts{};
    uint64_t budget = 0;
    uint32_t max_slots = 0;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    std::map<Instance *, Request *> running;
    bool stop = false;
    uint64_t next_ticket = 1;
    uint64_t in_use = 0;
    uint64_t slots_in_use[2] = {0, 0}, slot_cap = 0;  // running requests' pair slots per run, and their bound
    uint32_t count[2] = {0, 0};                         // running requests per run
    std::unique_ptr<Run> run[2];                        // small, large
    hipStream_t stream = nullptr;  // the worker's own stream (default priority): rounds are
                                   // captured on it, so callers' use of the context's
                                   // stream (readout, frees) never meets a capture
    std::string fatal;

    void loop();
    bool step(Run &r);
};

// Rounds of one run, then its converged (or round-limited) instances handed
// back.  false: a device failure ended every request.
bool cflr_server::step(Run &rn) {
    try {
        rn.rounds(opts.rounds_per_sync ? opts.rounds_per_sync : 2);
        std::vector<std::shared_ptr<Instance>> done;
        for (auto &ip : rn.instances())
            if (ip->done || (opts.max_rounds && ip->rounds >= opts.max_rounds)) done.push_back(ip);
        for (auto &ip : done) {
            rn.remove(ip.get());
            ip->stats.rounds = ip->rounds;
            ip->stats.reruns = rn.reruns();
            cflr_status st = ip->done ? CFLR_OK : CFLR_ETIMEOUT;
            compact_instance(*ip);
            instance_counts(*ip);
            std::lock_guard<std::mutex> lk(mu);
            Request *r = running[ip.get()];
            running.erase(ip.get());
            in_use -= r->footprint;
            slots_in_use[r->cls] -= r->slots;
            count[r->cls]--;
            r->status = st;
            if (st != CFLR_OK) r->error = "round limit reached before the fixpoint";
            r->t_finish = now_s();
            r->inst->stats.fixpoint_ms = (r->t_finish - r->t_admit) * 1e3;
            r->finished = true;
        }
        if (!done.empty()) cv_done.notify_all();
        return true;
    } catch (const std::exception &e) {
        // a device failure ends every running request
        std::lock_guard<std::mutex> lk(mu);
        fatal = e.what();
        for (auto &kv : running) {
            kv.second->status = CFLR_EDEVICE;
            kv.second->error = fatal;
            kv.second->finished = true;
            kv.second->t_finish = now_s();
        }
        running.clear();
        for (Request *r : queue) {
            r->status = CFLR_EDEVICE;
            r->error = fatal;
            r->finished = true;
        }
        queue.clear();
        stop = true;
        cv_done.notify_all();
        return false;
    }
}

void cflr_server::loop() {
    (void)hipSetDevice(ctx->device);
    uint64_t batch = 0;
    while (true) {
        std::vector<Request *> admit;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !queue.empty() || !running.empty(); });
            if (stop && queue.empty() && running.empty()) break;
            uint64_t planned = in_use, planned_slots[2] = {slots_in_use[0], slots_in_use[1]};
            uint32_t planned_count[2] = {count[0], count[1]};
            for (auto it = queue.begin(); it != queue.end();) {
                Request *r = *it;
                if (r->footprint > budget) {
                    it = queue.erase(it);
                    r->status = CFLR_ENOMEM;
                    r->error = "request footprint exceeds the server budget";
                    r->finished = true;
                    r->t_finish = now_s();
                    cv_done.notify_all();
                    continue;
                }
                const int c = r->cls;
                // the pair-slot bound keeps one round's new pairs inside the
                // 2^32-entry buffer and a round short enough for latency
                const bool idle = planned_count[0] + planned_count[1] == 0;
                const bool fits = planned_count[c] < max_slots &&
                                  (idle || (planned + r->footprint <= budget &&
                                            (planned_count[c] == 0 || planned_slots[c] + r->slots <= slot_cap)));
                if (!fits) {
                    ++it;
                    continue;
                }
                it = queue.erase(it);
                admit.push_back(r);
                planned += r->footprint;
                planned_slots[c] += r->slots;
                planned_count[c]++;
            }
        }
        for (Request *r : admit) {
            try {
                auto inst = make_instance(ctx, r->g->low, r->graph);
                run[r->cls]->add(inst);
                std::lock_guard<std::mutex> lk(mu);
                r->inst = inst;
                r->t_admit = now_s();
                running[inst.get()] = r;
                in_use += r->footprint;
                slots_in_use[r->cls] += r->slots;
                count[r->cls]++;
            } catch (const Error &e) {
                std::lock_guard<std::mutex> lk(mu);
                if (e.status == CFLR_ENOMEM && !running.empty()) {
                    queue.push_front(r);  // wait for memory to free up
                } else {
                    r->status = e.status;
                    r->error = e.what();
                    r->finished = true;
                    r->t_finish = now_s();
                    cv_done.notify_all();
                }
            }
        }
        const bool small = run[0]->size() > 0, large = run[1]->size() > 0;
        if (!small && !large) continue;
        if (small && !step(*run[0])) break;
        if (large && (!small || batch % kSmallPace == 0) && !step(*run[1])) break;
        batch++;
    }
}

extern "C" {

static cflr_status server_fail(cflr_status st, const std::string &msg) {
    set_last_error(msg);
    return st;
}

cflr_status cflr_server_create(cflr_ctx *ctx, uint64_t hbm_budget_bytes, uint32_t max_slots,
                               const cflr_opts *opts, cflr_server **out) {
    set_last_error("");
    if (!ctx || !out) return server_fail(CFLR_EINVAL, "null argument");
    if (!max_slots) return server_fail(CFLR_EINVAL, "max_slots must be at least 1");
    if (opts && opts->witness) return server_fail(CFLR_EUNSUPPORTED, "served requests record no witnesses");
    *out = nullptr;
    try {
        hip_check(hipSetDevice(ctx->device), "hipSetDevice");
        auto s = std::make_unique<cflr_server>();
        s->hold = CtxRef(ctx);
        s->ctx = ctx;
        cflr_opts_default(&s->opts);
        if (opts) s->opts = *opts;
        s->budget = hbm_budget_bytes;
        s->slot_cap = std::min<uint64_t>(1ull << 29, std::max<uint64_t>(1ull << 20, hbm_budget_bytes / 16));
        s->max_slots = max_slots;
        // sort buckets: an instance needs far less than 1/65536 of its
        // footprint in buckets (one per key tile and 4096-partner segment of
        // a sorted matrix); capped at 2^26.  The large run's new-pair buffer
        // starts at the size earlier solves on ctx grew it to (else 2^26
        // pairs), at most a budget's worth (44 bytes a pair), the small
        // run's at 2^22 pairs at most, unless the options say otherwise
        // (both grow on overflow).
        uint64_t buckets = std::min<uint64_t>(1ull << 26, std::max<uint64_t>(1ull << 20, hbm_budget_bytes / 65536));
        cflr_opts o_run[2] = {s->opts, s->opts};
        if (!s->opts.delta_capacity) {
            const uint64_t want = ctx->delta_capacity_hint ? ctx->delta_capacity_hint : 1ull << 26;
            o_run[1].delta_capacity = std::max<uint64_t>(1ull << 20, std::min(want, hbm_budget_bytes / 44));
            o_run[0].delta_capacity = std::min<uint64_t>(o_run[1].delta_capacity, 1ull << 22);
        }
        hip_check(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "hipStreamCreate");
        try {
            for (int c = 0; c < 2; c++)
                s->run[c] = std::make_unique<Run>(ctx, o_run[c], buckets, max_slots, s->stream);
        } catch (...) {
            for (auto &rn : s->run) rn.reset();
            (void)hipStreamDestroy(s->stream);
            throw;
        }
        s->worker = std::thread([p = s.get()] { p->loop(); });
        *out = s.release();
        return CFLR_OK;
    } catch (const Error &e) {
        return server_fail(e.status, e.what());
    } catch (const std::bad_alloc &) {
        return server_fail(CFLR_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return server_fail(CFLR_EDEVICE, e.what());
    }
}

cflr_status cflr_server_submit(cflr_server *s, const cflr_grammar *g, const cflr_graph *graph, uint64_t *ticket) {
    set_last_error("");
    if (!s || !g || !graph || !ticket) return server_fail(CFLR_EINVAL, "null argument");
    if (graph->ctx != s->ctx) return server_fail(CFLR_EINVAL, "graph belongs to another context");
    auto r = std::make_unique<Request>();
    r->g = g;
    r->graph = graph;
    r->t_submit = now_s();
    r->footprint = instance_footprint(g->low, graph->n);
    r->slots = instance_pair_slots(g->low, graph->n);
    r->cls = r->footprint <= s->budget / kSmallShare ? 0 : 1;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return server_fail(CFLR_EDEVICE, "server stopped: " + s->fatal);
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->queue.push_back(r.get());
    s->reqs[r->ticket] = std::move(r);
    s->cv_work.notify_one();
    return CFLR_OK;
}

static cflr_status take(cflr_server *s, Request *r, cflr_result **out) {
    if (r->taken) return server_fail(CFLR_EINVAL, "result of this ticket already taken");
    r->taken = true;
    if (r->status != CFLR_OK) set_last_error(r->error);
    if (r->status != CFLR_OK && r->status != CFLR_ETIMEOUT) return r->status;
    *out = new cflr_result{r->inst};
    (void)s;
    return r->status;
}

cflr_status cflr_server_poll(cflr_server *s, uint64_t ticket, cflr_result **out) {
    set_last_error("");
    if (!s || !out) return server_fail(CFLR_EINVAL, "null argument");
    *out = nullptr;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return server_fail(CFLR_EINVAL, "unknown ticket");
    if (!it->second->finished) return CFLR_PENDING;
    return take(s, it->second.get(), out);
}

cflr_status cflr_server_wait(cflr_server *s, uint64_t ticket, uint64_t timeout_ns, cflr_result **out) {
    set_last_error("");
    if (!s || !out) return server_fail(CFLR_EINVAL, "null argument");
    *out = nullptr;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return server_fail(CFLR_EINVAL, "unknown ticket");
    Request *r = it->second.get();
    bool ok = s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), [&] { return r->finished; });
    if (!ok) return server_fail(CFLR_ETIMEOUT, "request not finished within the timeout");
    return take(s, r, out);
}

cflr_status cflr_server_times(cflr_server *s, uint64_t ticket, double *submitted, double *admitted,
                              double *finished) {
    set_last_error("");
    if (!s) return server_fail(CFLR_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return server_fail(CFLR_EINVAL, "unknown ticket");
    Request *r = it->second.get();
    if (!r->finished) return server_fail(CFLR_PENDING, "request not finished");
    if (submitted) *submitted = r->t_submit;
    if (admitted) *admitted = r->t_admit;
    if (finished) *finished = r->t_finish;
    return CFLR_OK;
}

void cflr_server_free(cflr_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto &rn : s->run) rn.reset();
    if (s->stream) {
        (void)hipSetDevice(s->ctx->device);
        (void)hipStreamSynchronize(s->stream);
        (void)hipStreamDestroy(s->stream);
    }
    delete s;
}

}  // extern "C"

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
//
// A request whose dense matrices would not fit the budget goes to a lane of
// its own: a second thread solves such requests
// one at a time on the sparse engine (memory proportional to the pairs, not
// counted in the budget), on its own stream, beside the two runs.  When the
// running instances of a run derive more new pairs in one round than the
// dense engine's buffer may hold (2^32), or its growth finds no memory, they
// go back to the front of the queue, start again from scratch, and that run
// admits at most half as many from then on; a request that cannot get its
// dense memory while nothing else holds any goes to the sparse lane.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
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
    int cls = 1;         // 0: small, 1: large, 2: the sparse lane
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
    uint32_t run_cap[2] = {0, 0};                       // most requests a run may hold
    cflr_opts run_opts[2];
    uint64_t buckets = 0;
    std::unique_ptr<Run> run[2];                        // small, large
    hipStream_t stream = nullptr;  // the worker's own stream (default priority): rounds are
                                   // captured on it, so callers' use of the context's
                                   // stream (readout, frees) never meets a capture
    // the sparse lane
    std::thread sparse_worker;
    std::condition_variable cv_sparse;
    std::deque<Request *> sparse_queue;
    Request *sparse_current = nullptr;
    hipStream_t sparse_stream = nullptr;
    // a request that found no memory beside a busy sparse lane waits for the
    // lane's request to end before the dense runs admit again
    bool wait_for_lane = false;
    std::string fatal;

    void loop();
    void sparse_loop();
    bool step(int c);
    void fail_all(const std::string &what);
    void renew_run(int c, bool small);
};

// Replace run c by a new one (small: its new-pair buffer starts at 2^22
// pairs at most; it grows on overflow); when the device has no memory for it
// now, run c stays empty and the worker loop tries again later.
void cflr_server::renew_run(int c, bool small) {
    run[c].reset();
    cflr_opts o = run_opts[c];
    if (small) o.delta_capacity = std::min<uint64_t>(o.delta_capacity, 1ull << 22);
    try {
        run[c] = std::make_unique<Run>(ctx, o, buckets, max_slots, stream);
    } catch (const Error &e) {
        if (e.status != CFLR_ENOMEM) throw;
        run[c].reset();
    }
}

// A device failure ends every request (callers hold the lock).
void cflr_server::fail_all(const std::string &what) {
    fatal = what;
    for (auto &kv : running) {
        kv.second->status = CFLR_EDEVICE;
        kv.second->error = fatal;
        kv.second->finished = true;
        kv.second->t_finish = now_s();
    }
    running.clear();
    for (auto *q : {&queue, &sparse_queue}) {
        for (Request *r : *q) {
            r->status = CFLR_EDEVICE;
            r->error = fatal;
            r->finished = true;
        }
        q->clear();
    }
    stop = true;
    cv_done.notify_all();
    cv_sparse.notify_all();
}

// Rounds of run c, then its converged (or round-limited) instances handed
// back.  false: a device failure ended every request.
bool cflr_server::step(int c) {
    Run &rn = *run[c];
    try {
        try {
            rn.rounds(opts.rounds_per_sync ? opts.rounds_per_sync : 2);
        } catch (const Error &e) {
            if (e.status != CFLR_ENOMEM) throw;
            // one round's new pairs passed the buffer's limit, or its growth
            // found no memory: the running requests start again (front of the
            // queue, in arrival order) and the run admits at most half as
            // many from now on; a request that ran alone goes to the sparse
            // lane unless the other run or the lane holds memory too
            std::lock_guard<std::mutex> lk(mu);
            std::vector<Request *> back;
            for (auto &ip : rn.instances()) {
                Request *r = running[ip.get()];
                running.erase(ip.get());
                in_use -= r->footprint;
                slots_in_use[c] -= r->slots;
                r->inst.reset();
                back.push_back(r);
            }
            std::sort(back.begin(), back.end(), [](Request *a, Request *b) { return a->ticket < b->ticket; });
            if (std::getenv("CFLR_PROGRESS"))
                std::fprintf(stderr, "[cflr] server: %s with %zu requests running; they start again, %zu at most\n",
                             e.what(), back.size(), std::max<size_t>(1, back.size() / 2));
            if (back.size() == 1 && running.empty() && !sparse_current) {
                // nothing else holds device memory: the sparse lane takes it
                // (its memory follows the pairs, not n^2)
                back[0]->cls = 2;
                sparse_queue.push_front(back[0]);
                cv_sparse.notify_one();
            } else {
                for (auto it = back.rbegin(); it != back.rend(); ++it) queue.push_front(*it);
                run_cap[c] = std::max<uint32_t>(1, (uint32_t)back.size() / 2);
                if (sparse_current && running.empty()) wait_for_lane = true;
            }
            count[c] = 0;
            renew_run(c, true);
            return true;
        }
        std::vector<std::shared_ptr<Instance>> done;
        for (auto &ip : rn.instances())
            if (ip->done || (opts.max_rounds && ip->rounds >= opts.max_rounds)) done.push_back(ip);
        for (auto &ip : done) {
            rn.remove(ip.get());
            ip->stats.rounds = ip->rounds;
            ip->stats.reruns = rn.reruns();
            ip->stats.storage = CFLR_STORAGE_DENSE;
            cflr_status st = ip->done ? CFLR_OK : CFLR_ETIMEOUT;
            std::string err = st == CFLR_OK ? "" : "round limit reached before the fixpoint";
            try {
                compact_instance(*ip);
                instance_counts(*ip);
            } catch (const Error &e) {
                if (e.status != CFLR_ENOMEM) throw;
                st = CFLR_ENOMEM;  // no memory for its readout tables: this request fails alone
                err = e.what();
            }
            std::lock_guard<std::mutex> lk(mu);
            Request *r = running[ip.get()];
            running.erase(ip.get());
            in_use -= r->footprint;
            slots_in_use[r->cls] -= r->slots;
            count[r->cls]--;
            r->status = st;
            r->error = err;
            r->t_finish = now_s();
            r->inst->stats.fixpoint_ms = (r->t_finish - r->t_admit) * 1e3;
            r->finished = true;
        }
        if (!done.empty()) {
            // an idle run whose new-pair buffer grew past a quarter of the
            // budget (44 bytes a pair) gives the memory back: a later large
            // request or the sparse lane may need it
            if (rn.size() == 0 && rn.delta_capacity() > run_opts[c].delta_capacity &&
                rn.delta_capacity() * 44 > budget / 4) {
                std::lock_guard<std::mutex> lk(mu);
                renew_run(c, false);
            }
            cv_done.notify_all();
        }
        return true;
    } catch (const std::exception &e) {
        std::lock_guard<std::mutex> lk(mu);
        fail_all(e.what());
        return false;
    }
}

// The sparse lane: one request at a time on the sparse engine.
void cflr_server::sparse_loop() {
    (void)hipSetDevice(ctx->device);
    while (true) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_sparse.wait(lk, [&] { return stop || !sparse_queue.empty(); });
            if (sparse_queue.empty()) break;
            r = sparse_queue.front();
            sparse_queue.pop_front();
            r->t_admit = now_s();
            sparse_current = r;
        }
        std::shared_ptr<Instance> inst;
        cflr_status st = CFLR_OK;
        std::string err;
        try {
            inst = make_instance(ctx, r->g->low, r->graph, false);
            bool timed_out = false;
            // structures start at 2^24 new pairs and grow with the request,
            // not at what the context's largest earlier solve grew them to
            cflr_opts lo = opts;
            if (!lo.delta_capacity) lo.delta_capacity = 1ull << 24;
            sparse_solve(ctx, lo, *inst, &timed_out, sparse_stream);
            inst->stats.storage = CFLR_STORAGE_SPARSE;
            instance_counts(*inst);
            if (timed_out) {
                st = CFLR_ETIMEOUT;
                err = "round limit reached before the fixpoint";
            }
        } catch (const Error &e) {
            st = e.status;
            err = e.what();
        } catch (const std::exception &e) {
            st = CFLR_EDEVICE;
            err = e.what();
        }
        std::unique_lock<std::mutex> lk(mu);
        sparse_current = nullptr;
        if (st == CFLR_ENOMEM && std::getenv("CFLR_PROGRESS"))
            std::fprintf(stderr, "[cflr] server: sparse lane request %llu: %s (%zu dense requests running)\n",
                         (unsigned long long)r->ticket, err.c_str(), running.size());
        if (st == CFLR_ENOMEM && !running.empty() && !stop) {
            // the dense runs hold the memory: try again once one of them retires
            inst.reset();
            sparse_queue.push_front(r);
            const size_t before = running.size();
            cv_done.notify_all();  // a dense admission may wait for this lane
            cv_done.wait(lk, [&] { return stop || running.size() < before; });
            continue;
        }
        r->status = st;
        r->error = err;
        if (st == CFLR_OK || st == CFLR_ETIMEOUT) r->inst = inst;
        r->t_finish = now_s();
        if (r->inst) r->inst->stats.fixpoint_ms = (r->t_finish - r->t_admit) * 1e3;
        r->finished = true;
        cv_done.notify_all();
    }
}

void cflr_server::loop() {
    (void)hipSetDevice(ctx->device);
    uint64_t batch = 0;
    while (true) {
        bool have[2] = {true, true};
        try {
            std::lock_guard<std::mutex> lk(mu);
            for (int c = 0; c < 2; c++) {
                if (!run[c]) renew_run(c, true);
                have[c] = run[c] != nullptr;
            }
        } catch (const std::exception &e) {
            std::lock_guard<std::mutex> lk(mu);
            fail_all(e.what());
            break;
        }
        if (!have[0] || !have[1]) {
            // no memory for a run yet: while nothing runs, wait a little for
            // the sparse lane or a retirement to free some
            std::unique_lock<std::mutex> lk(mu);
            if (running.empty()) cv_done.wait_for(lk, std::chrono::milliseconds(20));
        }
        std::vector<Request *> admit;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (wait_for_lane) {
                cv_done.wait(lk, [&] { return stop || !sparse_current; });
                wait_for_lane = false;
            }
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
                const bool fits = have[c] && planned_count[c] < run_cap[c] &&
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
        bool wait_lane = false;
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
                if (e.status == CFLR_ENOMEM && (!running.empty() || sparse_current)) {
                    queue.push_front(r);  // wait for memory to free up
                    if (running.empty()) wait_lane = true;
                } else if (e.status == CFLR_ENOMEM) {
                    r->cls = 2;  // its dense matrices do not fit the device: the sparse lane
                    sparse_queue.push_front(r);
                    cv_sparse.notify_one();
                } else {
                    r->status = e.status;
                    r->error = e.what();
                    r->finished = true;
                    r->t_finish = now_s();
                    cv_done.notify_all();
                }
            }
        }
        if (wait_lane) {
            // only the sparse lane holds memory: wait until its request ends
            std::unique_lock<std::mutex> lk(mu);
            cv_done.wait(lk, [&] { return stop || !sparse_current || !running.empty(); });
        }
        const bool small = run[0] && run[0]->size() > 0, large = run[1] && run[1]->size() > 0;
        if (!small && !large) continue;
        if (small && !step(0)) break;
        if (large && (!small || batch % kSmallPace == 0) && !step(1)) break;
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
        // pairs), at most a quarter of the budget (44 bytes a pair), the small
        // run's at 2^22 pairs at most, unless the options say otherwise
        // (both grow on overflow).
        const uint64_t buckets = std::min<uint64_t>(1ull << 26, std::max<uint64_t>(1ull << 20, hbm_budget_bytes / 65536));
        s->buckets = buckets;
        s->run_cap[0] = s->run_cap[1] = max_slots;
        cflr_opts o_run[2] = {s->opts, s->opts};
        if (!s->opts.delta_capacity) {
            const uint64_t want = ctx->delta_capacity_hint ? ctx->delta_capacity_hint : 1ull << 26;
            o_run[1].delta_capacity = std::max<uint64_t>(1ull << 20, std::min(want, hbm_budget_bytes / 4 / 44));
            o_run[0].delta_capacity = std::min<uint64_t>(o_run[1].delta_capacity, 1ull << 22);
        }
        s->run_opts[0] = o_run[0];
        s->run_opts[1] = o_run[1];
        hip_check(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking), "hipStreamCreate");
        try {
            hip_check(hipStreamCreateWithFlags(&s->sparse_stream, hipStreamNonBlocking), "hipStreamCreate");
            for (int c = 0; c < 2; c++)
                s->run[c] = std::make_unique<Run>(ctx, o_run[c], buckets, max_slots, s->stream);
        } catch (...) {
            for (auto &rn : s->run) rn.reset();
            (void)hipStreamDestroy(s->stream);
            if (s->sparse_stream) (void)hipStreamDestroy(s->sparse_stream);
            throw;
        }
        s->worker = std::thread([p = s.get()] { p->loop(); });
        s->sparse_worker = std::thread([p = s.get()] { p->sparse_loop(); });
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
    r->cls = r->footprint <= s->budget / kSmallShare ? 0 : r->footprint <= s->budget ? 1 : 2;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return server_fail(CFLR_EDEVICE, "server stopped: " + s->fatal);
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    if (r->cls == 2) {
        s->sparse_queue.push_back(r.get());
        s->cv_sparse.notify_one();
    } else {
        s->queue.push_back(r.get());
        s->cv_work.notify_one();
    }
    s->reqs[r->ticket] = std::move(r);
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
        s->cv_sparse.notify_all();
        s->cv_done.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    if (s->sparse_worker.joinable()) s->sparse_worker.join();
    for (auto &rn : s->run) rn.reset();
    (void)hipSetDevice(s->ctx->device);
    for (hipStream_t st : {s->stream, s->sparse_stream}) {
        if (!st) continue;
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    delete s;
}

}  // extern "C"

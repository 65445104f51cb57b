// api.cpp -- the extern "C" boundary of libcflr (include/cflr.h).
//
// Every entry point catches C++ exceptions and turns them into a status plus
// a thread-local message; nothing throws across the boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <string>

#include "engine.h"

using namespace cflr;

namespace cflr {

// Free the column-major copies and the helper matrices of a finished
// instance, keeping only the row-major matrices of the user non-terminals
// that readout needs.
void compact_instance(Instance &in) {
    if (in.sp) return;  // sparse storage keeps only lists
    const uint32_t U = (uint32_t)in.low.user_names.size();
    const uint64_t words = (uint64_t)in.n * in.Wp;
    const uint64_t bytes = words * 8 * U;
    if (!bytes || bytes >= in.arena.bytes) return;
    DevBuf nb(in.ctx->pool.get(), bytes);
    uint64_t *p = nb.as<uint64_t>();
    std::vector<MatDev> mats(U);
    for (uint32_t x = 0; x < U; x++) {
        hip_check(hipMemcpyAsync(p, in.mats[x].R, (uint64_t)in.n * in.Wp * 8, hipMemcpyDeviceToDevice,
                                 in.ctx->stream),
                  "D2D");
        mats[x].R = p;
        mats[x].C = nullptr;
        mats[x].Rm = mats[x].Cm = nullptr;
        mats[x].sort = 0;
        mats[x].rrank = mats[x].crank = 0;
        p += words;
    }
    hip_check(hipStreamSynchronize(in.ctx->stream), "sync");
    in.arena = std::move(nb);
    in.mats = std::move(mats);
    in.stats.device_bytes = bytes;
}

void set_last_error(const std::string &msg);

void ctx_retain(cflr_ctx *ctx) { ctx->refs.fetch_add(1); }

void ctx_release(cflr_ctx *ctx) {
    if (ctx->refs.fetch_sub(1) != 1) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->pool.reset();
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

}  // namespace cflr

namespace {

thread_local std::string g_last_error;
std::atomic<uint64_t> g_grammar_serial{1};

cflr_status fail(cflr_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

}  // namespace

void cflr::set_last_error(const std::string &msg) { g_last_error = msg; }

namespace {

template <class F>
cflr_status guard(F &&f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const Error &e) {
        return fail(e.status, e.what());
    } catch (const std::bad_alloc &) {
        return fail(CFLR_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(CFLR_EDEVICE, e.what());
    }
}

void set_device(cflr_ctx *ctx) { hip_check(hipSetDevice(ctx->device), "hipSetDevice"); }

// Storage of a single solve: dense bit matrices while they take at most a
// quarter of the device memory, else pair storage (cflr_opts.storage).
bool use_sparse(cflr_ctx *ctx, const cflr_opts &o, const Lowered &low, uint32_t n) {
    if (o.witness) {
        // witnesses live in the sparse engine's pair set, and are named in the
        // grammar text's symbols (no hidden helpers)
        if (o.storage == CFLR_STORAGE_DENSE)
            throw Error(CFLR_EUNSUPPORTED, "witnesses are recorded by the sparse storage only");
        if (low.helpers) throw Error(CFLR_EUNSUPPORTED, "witnesses need right sides of at most two symbols");
        if (!o.semi_naive) throw Error(CFLR_EUNSUPPORTED, "sparse storage runs the semi-naive rounds only");
        return true;
    }
    if (o.storage == CFLR_STORAGE_SPARSE) {
        if (!o.semi_naive) throw Error(CFLR_EUNSUPPORTED, "sparse storage runs the semi-naive rounds only");
        return true;
    }
    if (!o.semi_naive) return false;
    if (o.storage == CFLR_STORAGE_DENSE) return false;
    if (o.storage != CFLR_STORAGE_AUTO) throw Error(CFLR_EINVAL, "unknown storage option");
    size_t f = 0, t = 0;
    hip_check(hipMemGetInfo(&f, &t), "hipMemGetInfo");
    return instance_footprint(low, n) > (uint64_t)t / 4;
}

cflr_opts effective(const cflr_opts *o) {
    cflr_opts r;
    cflr_opts_default(&r);
    if (o) r = *o;
    return r;
}

}  // namespace

extern "C" {

void cflr_opts_default(cflr_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->semi_naive = 1;
}

const char *cflr_last_error(void) { return g_last_error.c_str(); }

const char *cflr_version(void) { return "cflr 0.1 gfx950"; }

// ------------------------------------------------------------------ context

cflr_status cflr_ctx_create(int hip_device, void *hip_stream, cflr_ctx **out) {
    return guard([&]() -> cflr_status {
        if (!out) return fail(CFLR_EINVAL, "out is null");
        *out = nullptr;
        int count = 0;
        hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount");
        if (hip_device < 0 || hip_device >= count)
            return fail(CFLR_EINVAL, "no HIP device " + std::to_string(hip_device));
        auto ctx = std::make_unique<cflr_ctx>();
        ctx->device = hip_device;
        hip_check(hipSetDevice(hip_device), "hipSetDevice");
        hipDeviceProp_t prop;
        hip_check(hipGetDeviceProperties(&prop, hip_device), "hipGetDeviceProperties");
        ctx->num_cu = (uint32_t)prop.multiProcessorCount;
        if (hip_stream) {
            ctx->stream = (hipStream_t)hip_stream;
        } else {
            hip_check(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking), "hipStreamCreate");
            ctx->own_stream = true;
        }
        ctx->pool = std::make_unique<DevPool>(hip_device);
        *out = ctx.release();
        return CFLR_OK;
    });
}

void cflr_ctx_destroy(cflr_ctx *ctx) {
    if (ctx) ctx_release(ctx);
}

cflr_status cflr_ctx_mem_info(cflr_ctx *ctx, uint64_t *free_bytes, uint64_t *total_bytes) {
    return guard([&]() -> cflr_status {
        if (!ctx || !free_bytes || !total_bytes) return fail(CFLR_EINVAL, "null argument");
        set_device(ctx);
        size_t f = 0, t = 0;
        hip_check(hipMemGetInfo(&f, &t), "hipMemGetInfo");
        *free_bytes = f;
        *total_bytes = t;
        return CFLR_OK;
    });
}

cflr_status cflr_ctx_trim(cflr_ctx *ctx) {
    return guard([&]() -> cflr_status {
        if (!ctx) return fail(CFLR_EINVAL, "null argument");
        set_device(ctx);
        hip_check(hipStreamSynchronize(ctx->stream), "sync");
        ctx->pool->trim();
        return CFLR_OK;
    });
}

// ------------------------------------------------------------------ grammar

cflr_status cflr_grammar_parse(const char *text, size_t len, cflr_grammar **out) {
    return guard([&]() -> cflr_status {
        if (!out || (!text && len)) return fail(CFLR_EINVAL, "null argument");
        *out = nullptr;
        auto g = std::make_unique<cflr_grammar>();
        g->low = parse_and_lower(text ? text : "", len);
        g->serial = g_grammar_serial++;
        *out = g.release();
        return CFLR_OK;
    });
}

void cflr_grammar_free(cflr_grammar *g) { delete g; }

uint32_t cflr_grammar_num_nonterminals(const cflr_grammar *g) {
    return g ? (uint32_t)g->low.user_names.size() : 0;
}

const char *cflr_grammar_nonterminal_name(const cflr_grammar *g, uint32_t nt) {
    if (!g || nt >= g->low.user_names.size()) return nullptr;
    return g->low.user_names[nt].c_str();
}

uint32_t cflr_grammar_num_terminals(const cflr_grammar *g) { return g ? (uint32_t)g->low.terminals.size() : 0; }

const char *cflr_grammar_terminal_name(const cflr_grammar *g, uint32_t t) {
    if (!g || t >= g->low.terminals.size()) return nullptr;
    return g->low.terminals[t].c_str();
}

cflr_status cflr_grammar_info_get(const cflr_grammar *g, cflr_grammar_info *out) {
    return guard([&]() -> cflr_status {
        if (!g || !out) return fail(CFLR_EINVAL, "null argument");
        out->user_nonterminals = (uint32_t)g->low.user_names.size();
        out->wrappers = g->low.wrappers;
        out->matrices = g->low.nmat();
        out->binary = (uint32_t)g->low.binary.size();
        out->terminal_rules = (uint32_t)g->low.term.size();
        out->eps_rules = (uint32_t)g->low.eps.size();
        out->terminals = (uint32_t)g->low.terminals.size();
        out->helpers = g->low.helpers;
        out->mirror_skipped = mirror_skipped(g->low);
        return CFLR_OK;
    });
}

// -------------------------------------------------------------------- graph

cflr_status cflr_graph_create(cflr_ctx *ctx, uint32_t n_vertices, uint64_t n_edges, const uint32_t *src,
                              const uint32_t *dst, const uint32_t *label, uint32_t n_labels,
                              const char *const *label_names, int on_device, cflr_graph **out) {
    return guard([&]() -> cflr_status {
        if (!ctx || !out) return fail(CFLR_EINVAL, "null argument");
        *out = nullptr;
        if (n_edges && (!src || !dst || !label)) return fail(CFLR_EINVAL, "null edge array");
        if (n_labels && !label_names) return fail(CFLR_EINVAL, "null label names");
        set_device(ctx);
        auto g = std::make_unique<cflr_graph>();
        g->hold = CtxRef(ctx);
        g->ctx = ctx;
        g->n = n_vertices;
        g->m = n_edges;
        for (uint32_t l = 0; l < n_labels; l++) {
            if (!label_names[l]) return fail(CFLR_EINVAL, "null label name");
            g->label_names.emplace_back(label_names[l]);
        }
        if (n_edges) {
            // validate on the host (device input is copied down first)
            std::vector<uint32_t> hs, hd, hl;
            const uint32_t *ps = src, *pd = dst, *pl = label;
            hipStream_t s = ctx->stream;
            if (on_device) {
                hs.resize(n_edges);
                hd.resize(n_edges);
                hl.resize(n_edges);
                copy_sync(hs.data(), src, n_edges * 4, hipMemcpyDeviceToHost, s);
                copy_sync(hd.data(), dst, n_edges * 4, hipMemcpyDeviceToHost, s);
                copy_sync(hl.data(), label, n_edges * 4, hipMemcpyDeviceToHost, s);
                ps = hs.data();
                pd = hd.data();
                pl = hl.data();
            }
            for (uint64_t e = 0; e < n_edges; e++) {
                if (ps[e] >= n_vertices || pd[e] >= n_vertices)
                    return fail(CFLR_EINVAL, "edge " + std::to_string(e) + " has a vertex >= n");
                if (pl[e] >= n_labels)
                    return fail(CFLR_EINVAL, "edge " + std::to_string(e) + " has a label >= n_labels");
            }
            DevPool *pool = ctx->pool.get();
            g->src = DevBuf(pool, n_edges * 4);
            g->dst = DevBuf(pool, n_edges * 4);
            g->lab = DevBuf(pool, n_edges * 4);
            copy_sync(g->src.ptr, ps, n_edges * 4, hipMemcpyHostToDevice, s);
            copy_sync(g->dst.ptr, pd, n_edges * 4, hipMemcpyHostToDevice, s);
            copy_sync(g->lab.ptr, pl, n_edges * 4, hipMemcpyHostToDevice, s);
        }
        *out = g.release();
        return CFLR_OK;
    });
}

void cflr_graph_free(cflr_graph *g) {
    if (!g) return;
    try {
        (void)hipSetDevice(g->ctx->device);
        (void)hipStreamSynchronize(g->ctx->stream);
    } catch (...) {
    }
    delete g;
}

// -------------------------------------------------------------------- solve

cflr_status cflr_solve(cflr_ctx *ctx, const cflr_grammar *g, const cflr_graph *graph, const cflr_opts *opts,
                       cflr_result **out) {
    return guard([&]() -> cflr_status {
        if (!ctx || !g || !graph || !out) return fail(CFLR_EINVAL, "null argument");
        if (graph->ctx != ctx) return fail(CFLR_EINVAL, "graph belongs to another context");
        *out = nullptr;
        set_device(ctx);
        cflr_opts o = effective(opts);
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        std::shared_ptr<Instance> inst;
        cflr_status status = CFLR_OK;
        const bool sparse = use_sparse(ctx, o, g->low, graph->n);
        if (sparse) {
            hip_check(hipEventRecord(e0, ctx->stream), "event");
            inst = make_instance(ctx, g->low, graph, false);
            bool timed_out = false;
            sparse_solve(ctx, o, *inst, &timed_out);
            if (timed_out) status = CFLR_ETIMEOUT;
            hip_check(hipEventRecord(e1, ctx->stream), "event");
            hip_check(hipEventSynchronize(e1), "event");
            float ms = 0;
            hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
            inst->stats.fixpoint_ms = ms;
            inst->stats.storage = CFLR_STORAGE_SPARSE;
        } else {
            hip_check(hipEventRecord(e0, ctx->stream), "event");
            inst = make_instance(ctx, g->low, graph);
            Run run(ctx, o, instance_buckets(g->low, graph->n), 1);
            run.add(inst);
            while (run.round()) {
                if (o.max_rounds && inst->rounds >= o.max_rounds) {
                    status = CFLR_ETIMEOUT;
                    break;
                }
            }
            hip_check(hipEventRecord(e1, ctx->stream), "event");
            hip_check(hipEventSynchronize(e1), "event");
            float ms = 0;
            hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
            inst->stats.fixpoint_ms = ms;
            inst->stats.rounds = inst->rounds;
            inst->stats.product_ms = run.product_ms();
            inst->stats.product_launches = run.product_launches();
            inst->stats.algo_bytes = run.algo_bytes();
            inst->stats.reruns = run.reruns();
            inst->stats.storage = CFLR_STORAGE_DENSE;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        instance_counts(*inst);
        *out = new cflr_result{inst};
        if (status != CFLR_OK) return fail(status, "round limit reached before the fixpoint");
        return CFLR_OK;
    });
}

cflr_status cflr_solve_noalloc(cflr_ctx *ctx, const cflr_grammar *g, uint32_t n_vertices, uint64_t n_edges,
                               const uint32_t *src, const uint32_t *dst, const uint32_t *label, uint32_t n_labels,
                               const char *const *label_names, const cflr_opts *opts, uint32_t *out_src,
                               uint32_t *out_dst, uint64_t capacity, uint64_t *counts, cflr_stats *stats) {
    return guard([&]() -> cflr_status {
        if (!ctx || !g || !counts) return fail(CFLR_EINVAL, "null argument");
        if (n_edges && (!src || !dst || !label)) return fail(CFLR_EINVAL, "null edge array");
        if (n_labels && !label_names) return fail(CFLR_EINVAL, "null label names");
        std::vector<std::string> names;
        for (uint32_t l = 0; l < n_labels; l++) {
            if (!label_names[l]) return fail(CFLR_EINVAL, "null label name");
            names.emplace_back(label_names[l]);
        }
        set_device(ctx);
        cflr_opts o = effective(opts);
        if (o.witness) return fail(CFLR_EUNSUPPORTED, "the no-alloc solve records no witnesses");
        sparse_solve_noalloc(ctx, g->low, n_vertices, n_edges, src, dst, label, names, o, out_src, out_dst, capacity,
                             counts, stats);
        return CFLR_OK;
    });
}

cflr_status cflr_solve_batch(cflr_ctx *ctx, const cflr_grammar *const *grammars, const cflr_graph *const *graphs,
                             uint32_t count, const cflr_opts *opts, cflr_result **outs) {
    return guard([&]() -> cflr_status {
        if (!ctx || (count && (!grammars || !graphs || !outs))) return fail(CFLR_EINVAL, "null argument");
        for (uint32_t k = 0; k < count; k++) {
            outs[k] = nullptr;
            if (!grammars[k] || !graphs[k]) return fail(CFLR_EINVAL, "null grammar or graph");
            if (graphs[k]->ctx != ctx) return fail(CFLR_EINVAL, "graph belongs to another context");
        }
        if (!count) return CFLR_OK;
        set_device(ctx);
        cflr_opts o = effective(opts);
        if (o.storage == CFLR_STORAGE_SPARSE)
            return fail(CFLR_EUNSUPPORTED, "batched solves use dense storage only");
        if (o.witness) return fail(CFLR_EUNSUPPORTED, "batched solves record no witnesses");
        // admission by device memory: instances join as earlier ones finish
        size_t free_b = 0, total_b = 0;
        hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
        // sort buckets: room for every graph at once, capped (later graphs
        // wait for earlier ones to retire)
        uint64_t buckets = 0, max_buckets = 0;
        for (uint32_t k = 0; k < count; k++) {
            uint64_t b = instance_buckets(grammars[k]->low, graphs[k]->n);
            buckets += b;
            max_buckets = std::max(max_buckets, b);
        }
        buckets = std::min<uint64_t>(buckets, std::max<uint64_t>(max_buckets, 0x0FFFFFFFull));
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        hip_check(hipEventRecord(e0, ctx->stream), "event");
        auto run = std::make_unique<Run>(ctx, o, buckets, count);
        // device memory for matrices: 70 % of what is free, minus the
        // new-pair buffer (44 bytes a pair: the append, two sort stages and
        // two sorted orders; grown on overflow) and headroom for it to
        // double once
        const uint64_t avail = (uint64_t)((double)(free_b + ctx->pool->held()) * 0.7);
        const uint64_t delta_bytes = 3 * 44ull * run->delta_capacity();
        const uint64_t budget = avail > delta_bytes ? avail - delta_bytes : avail / 4;
        std::vector<std::shared_ptr<Instance>> all(count);
        uint64_t in_use = 0;
        cflr_status status = CFLR_OK;
        std::vector<uint64_t> fp(count), wt(count);
        uint64_t max_wt = 0;
        for (uint32_t k = 0; k < count; k++) {
            fp[k] = instance_footprint(grammars[k]->low, graphs[k]->n);
            wt[k] = instance_pair_slots(grammars[k]->low, graphs[k]->n);
            max_wt = std::max(max_wt, wt[k]);
        }
        // running instances: their (key tile, partner) slots sum to at most this
        const uint64_t wt_cap = std::max<uint64_t>(max_wt, 0x0FFFFFFFull);
        uint64_t wt_in = 0;
        const bool progress = std::getenv("CFLR_PROGRESS") != nullptr;
        uint32_t finished = 0;
        // graphs waiting for admission, in order; a round whose new pairs
        // pass the buffer's 2^32 limit with several graphs running sends the
        // running ones back here (from scratch) and halves how many may run
        std::deque<uint32_t> waiting;
        for (uint32_t k = 0; k < count; k++) waiting.push_back(k);
        std::vector<uint8_t> retired(count, 0);
        // a context that had to restart a batch's graphs starts later batches
        // at the concurrency that fitted
        uint32_t max_running = ctx->batch_running_cap ? std::min(count, ctx->batch_running_cap) : count;
        const auto t_batch = std::chrono::steady_clock::now();
        double product_ms = 0;
        uint64_t launches = 0, algo = 0, reruns = 0;
        auto fold_run_stats = [&]() {
            product_ms += run->product_ms();
            launches += run->product_launches();
            algo += run->algo_bytes();
            reruns += run->reruns();
        };
        while (true) {
            // admit
            while (!waiting.empty() && run->size() < max_running) {
                const uint32_t k = waiting.front();
                const uint64_t need = fp[k];
                if (run->size() && (in_use + need > budget || wt_in + wt[k] > wt_cap)) break;
                auto inst = make_instance(ctx, grammars[k]->low, graphs[k]);
                try {
                    run->add(inst);
                } catch (const Error &e) {
                    if (!run->size()) throw;
                    break;  // bucket space full: wait for a retirement
                }
                all[k] = inst;
                in_use += need;
                wt_in += wt[k];
                waiting.pop_front();
            }
            if (!run->size()) break;
            try {
                run->rounds(o.rounds_per_sync ? o.rounds_per_sync
                                              : (ctx->rounds_per_sync_tuned ? ctx->rounds_per_sync_tuned : 4));
            } catch (const Error &e) {
                if (e.status != CFLR_ENOMEM || run->size() < 2) throw;
                // restart the running graphs in a new run with at most half as many at once
                std::vector<uint32_t> back;
                for (uint32_t k = 0; k < count; k++)
                    if (all[k] && !retired[k]) back.push_back(k);
                if (progress)
                    std::fprintf(stderr,
                                 "[cflr] batch: %s with %zu graphs running after %.2f s; they start again, %zu at most\n",
                                 e.what(), back.size(),
                                 std::chrono::duration<double>(std::chrono::steady_clock::now() - t_batch).count(),
                                 std::max<size_t>(1, back.size() / 2));
                max_running = std::max<uint32_t>(1, (uint32_t)back.size() / 2);
                ctx->batch_running_cap = max_running;
                fold_run_stats();
                run.reset();
                for (auto it = back.rbegin(); it != back.rend(); ++it) {
                    all[*it].reset();
                    waiting.push_front(*it);
                }
                in_use = wt_in = 0;
                cflr_opts ro = o;
                if (!ro.delta_capacity) ro.delta_capacity = 1ull << 28;  // not the limit the last run reached
                run = std::make_unique<Run>(ctx, ro, buckets, count);
                continue;
            }
            // retire finished instances
            std::vector<std::shared_ptr<Instance>> done;
            for (auto &ip : run->instances())
                if (ip->done || (o.max_rounds && ip->rounds >= o.max_rounds)) done.push_back(ip);
            for (auto &ip : done) {
                if (!ip->done) {
                    ip->status = CFLR_ETIMEOUT;
                    status = CFLR_ETIMEOUT;
                }
                run->remove(ip.get());
                in_use -= ip->footprint;
                wt_in -= instance_pair_slots(ip->low, ip->n);
                ip->stats.rounds = ip->rounds;
                compact_instance(*ip);
                for (uint32_t k = 0; k < count; k++)
                    if (all[k].get() == ip.get()) retired[k] = 1;
            }
            finished += (uint32_t)done.size();
            if (progress && !done.empty())
                std::fprintf(stderr, "[cflr] batch: %u of %u graphs done, %zu running\n", finished, count,
                             run->size());
        }
        fold_run_stats();
        hip_check(hipEventRecord(e1, ctx->stream), "event");
        hip_check(hipEventSynchronize(e1), "event");
        float ms = 0;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        for (uint32_t k = 0; k < count; k++) {
            Instance &in = *all[k];
            in.stats.fixpoint_ms = ms;  // the whole batch shares one clock
            in.stats.product_ms = product_ms;
            in.stats.product_launches = launches;
            in.stats.algo_bytes = algo;
            in.stats.reruns = reruns;
            in.stats.storage = CFLR_STORAGE_DENSE;
            instance_counts(in);
            outs[k] = new cflr_result{all[k]};
        }
        if (status != CFLR_OK) return fail(status, "round limit reached before the fixpoint");
        return CFLR_OK;
    });
}

cflr_status cflr_autotune(cflr_ctx *ctx, const cflr_grammar *const *grammars, const cflr_graph *const *graphs,
                          uint32_t count, uint32_t *out_grid_waves, uint32_t *out_rounds_per_sync,
                          double *out_best_ms) {
    return guard([&]() -> cflr_status {
        if (!ctx || !count || !grammars || !graphs) return fail(CFLR_EINVAL, "null argument");
        set_device(ctx);
        const bool verbose = std::getenv("CFLR_TUNE_LOG") != nullptr;
        std::vector<cflr_result *> outs(count, nullptr);
        uint32_t storage = 0;  // the engine the first trial ran on
        // one timed solve (or batch) with these options
        auto trial = [&](const cflr_opts &o, double *ms_out) -> cflr_status {
            hipEvent_t e0, e1;
            hip_check(hipEventCreate(&e0), "event");
            hip_check(hipEventCreate(&e1), "event");
            hip_check(hipEventRecord(e0, ctx->stream), "event");
            cflr_status st = count > 1 ? cflr_solve_batch(ctx, grammars, graphs, count, &o, outs.data())
                                       : cflr_solve(ctx, grammars[0], graphs[0], &o, outs.data());
            hip_check(hipEventRecord(e1, ctx->stream), "event");
            hip_check(hipEventSynchronize(e1), "event");
            float ms = 0;
            hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            if (st == CFLR_OK && outs[0] && !storage) storage = outs[0]->inst->stats.storage;
            for (auto &r : outs) {
                cflr_result_free(r);
                r = nullptr;
            }
            if (verbose && st == CFLR_OK)
                std::fprintf(stderr,
                             "[cflr] autotune grid_waves=%u rounds_per_sync=%u chunk_pairs=%u sparse_heavy=%u: %.1f ms\n",
                             o.grid_waves, o.rounds_per_sync, o.chunk_pairs, o.sparse_heavy, ms);
            *ms_out = ms;
            return st;
        };
        cflr_opts best;
        cflr_opts_default(&best);
        best.grid_waves = 32 * ctx->num_cu;
        best.rounds_per_sync = count > 1 ? 4 : 1;
        double best_ms = 1e300;
        // sweep one field over its candidates, the others at the best so far
        auto sweep = [&](uint32_t cflr_opts::*field, const std::vector<uint32_t> &cands) -> cflr_status {
            for (uint32_t v : cands) {
                cflr_opts o = best;
                o.*field = v;
                double ms = 0;
                cflr_status st = trial(o, &ms);
                if (st != CFLR_OK) return st;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = o;
                }
            }
            return CFLR_OK;
        };
        cflr_status st = sweep(&cflr_opts::grid_waves, {16 * ctx->num_cu, 32 * ctx->num_cu, 48 * ctx->num_cu});
        if (st == CFLR_OK && count > 1) st = sweep(&cflr_opts::rounds_per_sync, {2, 4, 8});
        if (st == CFLR_OK && storage == CFLR_STORAGE_DENSE)
            st = sweep(&cflr_opts::chunk_pairs, {1u << 18, 1u << 20, 1u << 22});
        if (st == CFLR_OK && storage == CFLR_STORAGE_SPARSE) st = sweep(&cflr_opts::sparse_heavy, {64, 128, 256});
        if (st != CFLR_OK) return st;
        ctx->grid_waves_tuned = best.grid_waves;
        ctx->rounds_per_sync_tuned = best.rounds_per_sync;
        // the defaults a trial left at 0 are kept as what they stand for
        if (storage == CFLR_STORAGE_DENSE) ctx->chunk_pairs_tuned = best.chunk_pairs ? best.chunk_pairs : kChunkPairs;
        if (storage == CFLR_STORAGE_SPARSE) ctx->sparse_heavy_tuned = best.sparse_heavy ? best.sparse_heavy : 128;
        if (out_grid_waves) *out_grid_waves = best.grid_waves;
        if (out_rounds_per_sync) *out_rounds_per_sync = best.rounds_per_sync;
        if (out_best_ms) *out_best_ms = best_ms;
        return CFLR_OK;
    });
}

cflr_status cflr_ctx_tuned(const cflr_ctx *ctx, cflr_opts *out) {
    return guard([&]() -> cflr_status {
        if (!ctx || !out) return fail(CFLR_EINVAL, "null argument");
        cflr_opts_default(out);
        out->grid_waves = ctx->grid_waves_tuned;
        out->rounds_per_sync = ctx->rounds_per_sync_tuned;
        out->chunk_pairs = ctx->chunk_pairs_tuned;
        out->sparse_heavy = ctx->sparse_heavy_tuned;
        return CFLR_OK;
    });
}

// ------------------------------------------------------------------ results

cflr_status cflr_result_count(const cflr_result *r, uint32_t nt, uint64_t *n_pairs) {
    return guard([&]() -> cflr_status {
        if (!r || !n_pairs) return fail(CFLR_EINVAL, "null argument");
        Instance &in = *r->inst;
        if (nt >= in.low.user_names.size()) return fail(CFLR_EINVAL, "non-terminal index out of range");
        set_device(in.ctx);
        instance_counts(in);
        *n_pairs = (uint64_t)in.counts[nt];
        return CFLR_OK;
    });
}

cflr_status cflr_result_copy(const cflr_result *r, uint32_t nt, uint32_t *src, uint32_t *dst, uint64_t capacity,
                             int on_device, uint64_t *written) {
    return guard([&]() -> cflr_status {
        if (!r || !written) return fail(CFLR_EINVAL, "null argument");
        Instance &in = *r->inst;
        if (nt >= in.low.user_names.size()) return fail(CFLR_EINVAL, "non-terminal index out of range");
        set_device(in.ctx);
        instance_counts(in);
        if (in.counts[nt] > 0 && (!src || !dst)) return fail(CFLR_EINVAL, "null output array");
        instance_copy(in, nt, src, dst, capacity, on_device != 0, written);
        return CFLR_OK;
    });
}

cflr_status cflr_result_witness(const cflr_result *r, uint32_t nt, uint32_t *left, uint32_t *right, uint32_t *mid,
                                uint32_t *round, uint64_t capacity, int on_device, uint64_t *written) {
    return guard([&]() -> cflr_status {
        if (!r || !written) return fail(CFLR_EINVAL, "null argument");
        Instance &in = *r->inst;
        if (nt >= in.low.user_names.size()) return fail(CFLR_EINVAL, "non-terminal index out of range");
        if (!in.sp || !in.sp->hash_slots) return fail(CFLR_EINVAL, "no witnesses: solve with cflr_opts.witness = 1");
        set_device(in.ctx);
        instance_counts(in);
        const uint64_t count = (uint64_t)in.counts[nt];
        if (capacity < count) return fail(CFLR_EINVAL, "capacity smaller than the pair count");
        if (count && (!left || !right || !mid || !round)) return fail(CFLR_EINVAL, "null output array");
        sparse_witness(in, nt, left, right, mid, round, count, on_device != 0);
        *written = count;
        return CFLR_OK;
    });
}

cflr_status cflr_result_stats(const cflr_result *r, cflr_stats *out) {
    return guard([&]() -> cflr_status {
        if (!r || !out) return fail(CFLR_EINVAL, "null argument");
        *out = r->inst->stats;
        return CFLR_OK;
    });
}

void cflr_result_free(cflr_result *r) {
    if (!r) return;
    try {
        (void)hipSetDevice(r->inst->ctx->device);
        (void)hipStreamSynchronize(r->inst->ctx->stream);
    } catch (...) {
    }
    delete r;
}

}  // extern "C"

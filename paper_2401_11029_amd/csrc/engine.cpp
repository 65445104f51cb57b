// engine.cpp -- host side of the round engine.
//
// The fixpoint of Algorithm 1 in its semi-naive form (Section 3, opt. 1):
//   seed      edges and eps rules set the first pairs; they are the first
//             round's new pairs (M_old = empty);
//   round     sort of the appended new pairs by (key tile, partner) into
//             row and column order (this round's dA, dB) -> prep (work
//             table) -> product (every production and admitted instance;
//             one launch for the row parts, then one for the column parts)
//             -> fold of the new-pair counts;
//   converge  an instance whose round derived no pair is done (its new-pair
//             set is empty, so no later round can derive anything for it).
// If the new-pair buffer overflows, the product leaves the overflowing
// candidates out of M; the host grows the buffer and re-runs the product of
// the same round (OR is idempotent, so pairs already added are not found
// again and the missing ones are).
#include "engine.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

namespace cflr {

void hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    cflr_status st = (e == hipErrorOutOfMemory) ? CFLR_ENOMEM : CFLR_EDEVICE;
    throw Error(st, std::string(what) + ": " + hipGetErrorString(e));
}

// Stream-ordered copy that returns once the data has landed.
void copy_sync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s) {
    if (!bytes) return;
    hip_check(hipMemcpyAsync(dst, src, bytes, kind, s), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

// ------------------------------------------------------------------ DevPool

static size_t round_bytes(size_t b) {
    // small blocks: next power of two (>= 256 B); large: 2 MiB granules
    if (b < ((size_t)1 << 20)) {
        size_t r = 256;
        while (r < b) r <<= 1;
        return r;
    }
    const size_t g = (size_t)2 << 20;
    return (b + g - 1) / g * g;
}

DevPool::~DevPool() {
    (void)hipSetDevice(device_);
    for (auto &kv : cache_) (void)hipFree(kv.second);
    for (auto &kv : live_) (void)hipFree(kv.first);
}

void *DevPool::alloc(size_t bytes) {
    size_t b = round_bytes(bytes);
    std::lock_guard<std::mutex> g(mu_);
    auto it = cache_.find(b);
    if (it != cache_.end()) {
        void *p = it->second;
        cache_.erase(it);
        live_[p] = b;
        return p;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, b);
    if (e == hipErrorOutOfMemory && !cache_.empty()) {
        (void)hipGetLastError();
        for (auto &kv : cache_) {
            (void)hipFree(kv.second);
            held_ -= kv.first;
        }
        cache_.clear();
        e = hipMalloc(&p, b);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(e == hipErrorOutOfMemory ? CFLR_ENOMEM : CFLR_EDEVICE,
                    "hipMalloc(" + std::to_string(b) + "): " + hipGetErrorString(e));
    }
    live_[p] = b;
    held_ += b;
    return p;
}

void DevPool::release(void *p) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) return;
    cache_.insert({it->second, p});
    live_.erase(it);
}

void DevPool::trim() {
    std::lock_guard<std::mutex> g(mu_);
    for (auto &kv : cache_) {
        (void)hipFree(kv.second);
        held_ -= kv.first;
    }
    cache_.clear();
}

// ---------------------------------------------------------------- instances

static void plan_layout(const Lowered &low, uint32_t n, uint32_t *S, uint64_t *Wp,
                        std::vector<uint8_t> *has_col, uint64_t *bytes) {
    const uint64_t words = ((uint64_t)n + 63) / 64;
    *S = (uint32_t)std::max<uint64_t>(1, (words + kSegWords - 1) / kSegWords);
    *Wp = (uint64_t)*S * kSegWords;
    const uint64_t layout = (uint64_t)n * *Wp * 8;
    const uint64_t mask = (uint64_t)n * 8;  // one segment-mask word per row
    uint64_t total = 0;
    has_col->assign(low.nmat(), 0);
    for (uint32_t x = 0; x < low.nmat(); x++) {
        total += layout + mask;  // R
        if (low.dynamic[x] || low.slot_a[x]) {
            (*has_col)[x] = 1;
            total += layout + mask;
        }
    }
    *bytes = total;
}

uint64_t instance_footprint(const Lowered &low, uint32_t n) {
    uint32_t S;
    uint64_t Wp, bytes;
    std::vector<uint8_t> hc;
    plan_layout(low, n, &S, &Wp, &hc, &bytes);
    return bytes;
}

uint64_t instance_buckets(const Lowered &low, uint32_t n) {
    // the row-order and column-order counters share the instance's range:
    // it holds the larger of the two sets of sorted matrices, one bucket per
    // (key tile, partner segment)
    uint64_t rows = 0, cols = 0;
    for (uint32_t x = 0; x < low.nmat(); x++) {
        rows += low.slot_a[x] ? 1 : 0;
        cols += low.slot_b[x] ? 1 : 0;
    }
    const uint64_t segs = std::max<uint64_t>(1, ((uint64_t)n + kSegCols - 1) / kSegCols);
    return std::max(rows, cols) * key_tiles(n) * segs;
}

uint64_t instance_pair_slots(const Lowered &low, uint32_t n) {
    return (uint64_t)low.nmat() * key_tiles(n) * n;
}

std::shared_ptr<Instance> make_instance(cflr_ctx *ctx, const Lowered &low, const cflr_graph *g, bool dense) {
    if (low.nmat() > kMaxMats) throw Error(CFLR_EUNSUPPORTED, "grammar needs more than 65536 matrices");
    auto inst = std::make_shared<Instance>();
    inst->hold = CtxRef(ctx);
    inst->ctx = ctx;
    inst->low = low;
    inst->graph = g;
    inst->n = g->n;
    std::vector<uint8_t> has_col;
    uint64_t bytes;
    plan_layout(low, g->n, &inst->S, &inst->Wp, &has_col, &bytes);
    if (!dense) bytes = 0;
    // the product kernel addresses a matrix with 32-bit word offsets
    if (dense && (uint64_t)g->n * inst->Wp >= (1ull << 32))
        throw Error(CFLR_EUNSUPPORTED, "graph too large for dense bit matrices (n * row words >= 2^32)");
    inst->footprint = bytes;
    inst->counts.assign(low.user_names.size(), -1);
    const uint64_t layout_words = (uint64_t)g->n * inst->Wp;
    if (bytes) inst->arena = DevBuf(ctx->pool.get(), bytes);
    uint64_t *p = inst->arena.as<uint64_t>();
    inst->mats.resize(dense ? low.nmat() : 0);
    uint16_t rrank = 0, crank = 0;
    for (uint32_t x = 0; x < inst->mats.size(); x++) {
        MatDev &M = inst->mats[x];
        M.R = p;
        p += layout_words;
        M.C = nullptr;
        M.Rm = M.Cm = nullptr;
        M.sort = (low.slot_a[x] ? kSortRows : 0u) | (low.slot_b[x] ? kSortCols : 0u);
        M.rrank = low.slot_a[x] ? rrank++ : 0;
        M.crank = low.slot_b[x] ? crank++ : 0;
        if (has_col[x]) {
            M.C = p;
            p += layout_words;
        }
    }
    // the segment masks follow the matrices (every row start stays 512-byte aligned)
    for (uint32_t x = 0; x < inst->mats.size(); x++) {
        MatDev &M = inst->mats[x];
        M.Rm = p;
        p += g->n;
        if (M.C) {
            M.Cm = p;
            p += g->n;
        }
    }
    if (bytes) hip_check(hipMemsetAsync(inst->arena.ptr, 0, bytes, ctx->stream), "zero matrices");

    // graph label -> matrices x with x -> label (after lowering)
    std::map<std::string, uint32_t> term_id;
    for (uint32_t t = 0; t < low.terminals.size(); t++) term_id[low.terminals[t]] = t;
    std::vector<std::vector<uint32_t>> by_term(low.terminals.size());
    for (auto &tm : low.term) by_term[tm.first].push_back(tm.second);
    const uint32_t L = (uint32_t)g->label_names.size();
    std::vector<uint32_t> ptr(L + 1, 0), mats;
    uint32_t max_per_label = 0;
    for (uint32_t l = 0; l < L; l++) {
        auto it = term_id.find(g->label_names[l]);
        if (it != term_id.end())
            for (uint32_t x : by_term[it->second]) mats.push_back(x);
        ptr[l + 1] = (uint32_t)mats.size();
        max_per_label = std::max(max_per_label, ptr[l + 1] - ptr[l]);
    }
    inst->lm_ptr = DevBuf(ctx->pool.get(), ptr.size() * 4);
    copy_sync(inst->lm_ptr.ptr, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice, ctx->stream);
    inst->lm_mat = DevBuf(ctx->pool.get(), std::max<size_t>(1, mats.size()) * 4);
    if (!mats.empty())
        copy_sync(inst->lm_mat.ptr, mats.data(), mats.size() * 4, hipMemcpyHostToDevice, ctx->stream);
    inst->n_eps = (uint32_t)low.eps.size();
    inst->eps_mat = DevBuf(ctx->pool.get(), std::max<size_t>(1, low.eps.size()) * 4);
    if (!low.eps.empty())
        copy_sync(inst->eps_mat.ptr, low.eps.data(), low.eps.size() * 4, hipMemcpyHostToDevice, ctx->stream);
    inst->max_seeds = g->m * max_per_label + (uint64_t)g->n * inst->n_eps;
    inst->stats.device_bytes = bytes;
    return inst;
}

// ---------------------------------------------------------------------- Run

Run::Run(cflr_ctx *ctx, const cflr_opts &opts, uint64_t bucket_capacity, uint32_t max_instances, hipStream_t stream)
    : hold_(ctx), ctx_(ctx), opts_(opts), s_(stream ? stream : ctx->stream), bucket_cap_(bucket_capacity),
      max_inst_(max_instances) {
    if (bucket_cap_ >= 0xFFFFFFF0ull)
        throw Error(CFLR_EUNSUPPORTED, "too many sort buckets for one run (matrices x key tiles x segments >= 2^32)");
    if (max_inst_ == 0 || max_inst_ > kMaxSlots)
        throw Error(CFLR_EINVAL, "instances per run must be in [1, " + std::to_string(kMaxSlots) + "]");
    DevPool *pool = ctx->pool.get();
    free_buckets_[0] = bucket_cap_;
    d_rcnt_ = DevBuf(pool, (bucket_cap_ + 1) * 4);
    d_ccnt_ = DevBuf(pool, (bucket_cap_ + 1) * 4);
    d_bsum_ = DevBuf(pool, 2ull * scan_block_count(bucket_cap_) * 4);
    d_counters_ = DevBuf(pool, 64);
    d_inst_new_ = DevBuf(pool, (uint64_t)max_inst_ * kCountShards * 8);
    d_inst_over_ = DevBuf(pool, (uint64_t)max_inst_ * 4);
    d_active_ = DevBuf(pool, (uint64_t)max_inst_ * 4);
    d_slot_stats_ = DevBuf(pool, (uint64_t)max_inst_ * sizeof(SlotStats));
    hip_check(hipMemsetAsync(d_slot_stats_.ptr, 0, (uint64_t)max_inst_ * sizeof(SlotStats), s_), "memset");
    hip_check(hipMemsetAsync(d_counters_.ptr, 0, 64, s_), "memset");
    hip_check(hipMemsetAsync(d_inst_new_.ptr, 0, (uint64_t)max_inst_ * kCountShards * 8, s_), "memset");
    hip_check(hipMemsetAsync(d_inst_over_.ptr, 0, (uint64_t)max_inst_ * 4, s_), "memset");
    // the bucket starts must read as "no new pairs" before the first sort
    hip_check(launch_fill_u32(d_rcnt_.as<uint32_t>(), bucket_cap_ + 1, 0, s_), "fill");
    hip_check(launch_fill_u32(d_ccnt_.as<uint32_t>(), bucket_cap_ + 1, 0, s_), "fill");
    hip_check(hipHostMalloc((void **)&h_new_, (uint64_t)max_inst_ * 8, 0), "hipHostMalloc");
    hip_check(hipHostMalloc((void **)&h_over_, (uint64_t)max_inst_ * 4, 0), "hipHostMalloc");
    hip_check(hipHostMalloc((void **)&h_counters_, 64, 0), "hipHostMalloc");
    hip_check(hipHostMalloc((void **)&h_stats_, (uint64_t)max_inst_ * sizeof(SlotStats), 0), "hipHostMalloc");
    hip_check(hipEventCreate(&ev0_), "event");
    hip_check(hipEventCreate(&ev1_), "event");
    if (const char *l = std::getenv("CFLR_DENSE_PAIR_LIMIT"))
        ap_limit_ = std::max<uint64_t>(1024, std::min<uint64_t>(ap_limit_, std::strtoull(l, nullptr, 10)));
    uint64_t cap = opts_.delta_capacity ? opts_.delta_capacity : ctx->delta_capacity_hint;
    // first guess: an eighth of a pair per (key tile, partner) of the run
    if (!cap) cap = std::max<uint64_t>(1ull << 22, std::min<uint64_t>(bucket_cap_ * (kSegCols / 8), 1ull << 28));
    ensure_capacity(cap, false);
    log_ = std::getenv("CFLR_LOG") != nullptr;
    uint32_t waves = opts_.grid_waves ? opts_.grid_waves : ctx->grid_waves_tuned;
    if (!waves) waves = ctx->num_cu * 32;
    grid_ = std::max<uint32_t>(1, waves / kProdWaves);
}

Run::~Run() {
    if (h_new_) (void)hipHostFree(h_new_);
    if (h_over_) (void)hipHostFree(h_over_);
    if (h_counters_) (void)hipHostFree(h_counters_);
    if (h_stats_) (void)hipHostFree(h_stats_);
    if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
    if (ev0_) (void)hipEventDestroy(ev0_);
    if (ev1_) (void)hipEventDestroy(ev1_);
}

void Run::ensure_capacity(uint64_t pairs, bool keep) {
    if (pairs <= ap_cap_) return;
    const uint64_t limit = ap_limit_;
    if (ap_cap_ >= limit) throw Error(CFLR_ENOMEM, "new-pair buffer at its 2^32 limit");
    pairs = std::min(pairs, limit);
    DevPool *pool = ctx_->pool.get();
    DevBuf *bufs[7] = {&d_ap_key_, &d_ap_i_, &d_ap_j_, &d_rs_, &d_cs_, &d_rs_stage_, &d_cs_stage_};
    const size_t width[7] = {4, 4, 4, 8, 8, 8, 8};
    for (int q = 0; q < 7; q++) {
        DevBuf nb(pool, pairs * width[q]);
        if (keep && q < 5 && bufs[q]->ptr)
            hip_check(hipMemcpyAsync(nb.ptr, bufs[q]->ptr, ap_cap_ * width[q], hipMemcpyDeviceToDevice, s_),
                      "D2D");
        hip_check(hipStreamSynchronize(s_), "sync");
        *bufs[q] = std::move(nb);
    }
    ap_cap_ = pairs;
    generation_++;
    ctx_->delta_capacity_hint = std::max(ctx_->delta_capacity_hint, pairs);
}

uint64_t Run::alloc_buckets(uint64_t count) {
    for (auto it = free_buckets_.begin(); it != free_buckets_.end(); ++it) {
        if (it->second >= count) {
            uint64_t base = it->first, len = it->second;
            free_buckets_.erase(it);
            if (len > count) free_buckets_[base + count] = len - count;
            return base;
        }
    }
    throw Error(CFLR_ENOMEM, "run sort-bucket space exhausted");
}

void Run::free_buckets(uint64_t base, uint64_t count) {
    if (!count) return;
    auto it = free_buckets_.insert({base, count}).first;
    auto nx = std::next(it);
    if (nx != free_buckets_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        free_buckets_.erase(nx);
    }
    if (it != free_buckets_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            free_buckets_.erase(it);
        }
    }
}

void Run::add(const std::shared_ptr<Instance> &inst) {
    if (insts_.size() >= max_inst_) throw Error(CFLR_EINVAL, "run is full");
    const uint64_t nb = instance_buckets(inst->low, inst->n);
    const uint64_t base = alloc_buckets(nb);
    // slot: lowest index not used by a running instance
    std::vector<uint8_t> used(max_inst_, 0);
    for (auto &o : insts_) used[o->slot] = 1;
    uint32_t slot = 0;
    while (used[slot]) slot++;
    // The instance joins the run only once it is seeded: if a step throws
    // (ENOMEM growing the new-pair buffer, a device error), whatever it
    // appended is purged, its bucket range is released and the run is as
    // before, so the caller may retry it later.
    bool launched = false;
    try {
        inst->bbase = (uint32_t)base;
        inst->slot = slot;
        // seeds: appended after whatever is already waiting in the buffer
        hip_check(hipStreamSynchronize(s_), "sync");
        unsigned long long cur = 0;
        copy_sync(&cur, d_counters_.ptr, 8, hipMemcpyDeviceToHost, s_);
        ensure_capacity(cur + inst->max_seeds, true);
        hip_check(launch_fill_u64(d_inst_new_.as<unsigned long long>() + (uint64_t)slot * kCountShards, kCountShards,
                                  0, s_),
                  "fill");
        DevBuf dmats(ctx_->pool.get(), inst->mats.size() * sizeof(MatDev));
        hip_check(hipMemcpyAsync(dmats.ptr, inst->mats.data(), inst->mats.size() * sizeof(MatDev),
                                 hipMemcpyHostToDevice, s_),
                  "H2D");
        SeedArgs A{};
        A.mats = dmats.as<MatDev>();
        A.I = InstDev{inst->n, inst->S, inst->bbase, 0};
        A.inst = slot;
        A.src = inst->graph->src.as<uint32_t>();
        A.dst = inst->graph->dst.as<uint32_t>();
        A.lab = inst->graph->lab.as<uint32_t>();
        A.m = inst->graph->m;
        A.lm_ptr = inst->lm_ptr.as<uint32_t>();
        A.lm_mat = inst->lm_mat.as<uint32_t>();
        A.eps_mat = inst->eps_mat.as<uint32_t>();
        A.n_eps = inst->n_eps;
        A.ap_key = d_ap_key_.as<uint32_t>();
        A.ap_i = d_ap_i_.as<uint32_t>();
        A.ap_j = d_ap_j_.as<uint32_t>();
        A.ap_count = d_counters_.as<unsigned long long>();
        A.ap_cap = ap_cap_;
        A.inst_new = d_inst_new_.as<unsigned long long>();
        A.rcnt = d_rcnt_.as<uint32_t>();
        A.ccnt = d_ccnt_.as<uint32_t>();
        A.inst_overflow = d_inst_over_.as<uint32_t>();
        launched = true;
        hip_check(launch_seed(A, s_), "seed");
        hip_check(hipMemcpyAsync(h_new_ + slot, d_inst_new_.as<unsigned long long>() + (uint64_t)slot * kCountShards,
                                 8, hipMemcpyDeviceToHost, s_),
                  "D2H");
        hip_check(hipStreamSynchronize(s_), "sync");
    } catch (...) {
        if (launched) {
            (void)launch_purge_slot(d_ap_key_.as<uint32_t>(), d_counters_.as<unsigned long long>(), ap_cap_, slot,
                                    ctx_->num_cu * 4, s_);
            (void)launch_zero_counts(d_rcnt_.as<uint32_t>() + base, d_ccnt_.as<uint32_t>() + base, nb,
                                     reinterpret_cast<uint32_t *>(d_counters_.as<unsigned long long>() + 3), s_);
            (void)hipStreamSynchronize(s_);
        }
        free_buckets(base, nb);
        throw;
    }
    inst->stats.seed_pairs = h_new_[slot];
    inst->rounds = 0;
    inst->done = false;
    insts_.push_back(inst);
    dirty_ = true;
    // the seeds are not a round's new pairs; the slot's statistics start over
    hip_check(launch_fill_u64(d_inst_new_.as<unsigned long long>() + (uint64_t)slot * kCountShards, kCountShards, 0,
                              s_),
              "fill");
    hip_check(launch_fill_u32(reinterpret_cast<uint32_t *>(d_slot_stats_.as<SlotStats>() + slot),
                              sizeof(SlotStats) / 4, 0, s_),
              "fill");
}

uint64_t Run::bucket_hi() const {
    // buckets at or above the last free range's base are unused
    if (!free_buckets_.empty()) {
        auto last = std::prev(free_buckets_.end());
        if (last->first + last->second == bucket_cap_) return last->first;
    }
    return bucket_cap_;
}

void Run::remove(Instance *inst) {
    for (size_t k = 0; k < insts_.size(); k++) {
        if (insts_[k].get() == inst) {
            if (!inst->done) {
                // its pending pairs become holes, and the counts the flush
                // made for them leave its bucket range (which may be reused)
                hip_check(launch_purge_slot(d_ap_key_.as<uint32_t>(), d_counters_.as<unsigned long long>(),
                                            ap_cap_, inst->slot, ctx_->num_cu * 4, s_),
                          "purge");
                hip_check(launch_zero_counts(d_rcnt_.as<uint32_t>() + inst->bbase, d_ccnt_.as<uint32_t>() + inst->bbase,
                                             instance_buckets(inst->low, inst->n),
                                             reinterpret_cast<uint32_t *>(d_counters_.as<unsigned long long>() + 3), s_),
                          "zero counts");
            }
            free_buckets(inst->bbase, instance_buckets(inst->low, inst->n));
            insts_.erase(insts_.begin() + (long)k);
            dirty_ = true;
            return;
        }
    }
}

void Run::rebuild_tables() {
    if (!dirty_) return;
    DevPool *pool = ctx_->pool.get();
    std::vector<InstDev> hi;
    std::vector<MatDev> hm;
    std::vector<EntryDev> he;
    std::vector<uint64_t> toff;
    uint64_t tbits = 0;
    // instance table indexed by slot
    hi.assign(max_inst_, InstDev{0, 1, 0, 0});
    toff.assign(max_inst_, 0);
    for (auto &ip : insts_) {
        Instance &in = *ip;
        hi[in.slot] = InstDev{in.n, in.S, in.bbase, (uint32_t)hm.size()};
        for (auto &m : in.mats) hm.push_back(m);
        toff[in.slot] = tbits;
        tbits += (uint64_t)in.low.nmat() * 2 * in.n * in.S;
    }
    // entries: every row part (part 0) first, then every column part
    for (uint32_t part = 0; part < 2; part++)
        for (auto &ip : insts_)
            for (auto &b : ip->low.binary) he.push_back(EntryDev{ip->slot, b.c, b.a, b.b, part});
    nent_ = (uint32_t)he.size();
    // units: (entry, key tile); those of part 0 come first
    std::vector<UnitDev> hu;
    unit_split_ = 0;
    for (uint32_t e = 0; e < nent_; e++) {
        const InstDev &I = hi[he[e].inst];
        const uint32_t nt = key_tiles(I.n);
        const MatDev &op = hm[I.mat_off + (he[e].part == 0 ? he[e].a : he[e].b)];
        const uint32_t rank = he[e].part == 0 ? op.rrank : op.crank;
        for (uint32_t t = 0; t < nt; t++) hu.push_back(UnitDev{he[e], t, rank, 0, 0, I});
        if (he[e].part == 0) unit_split_ = (uint32_t)hu.size();
    }
    nunit_ = (uint32_t)hu.size();
    std::vector<uint32_t> active(max_inst_, 0);
    for (auto &ip : insts_) active[ip->slot] = 1;
    copy_sync(d_active_.ptr, active.data(), active.size() * 4, hipMemcpyHostToDevice, s_);
    generation_++;
    d_inst_ = DevBuf(pool, hi.size() * sizeof(InstDev));
    d_mats_ = DevBuf(pool, std::max<size_t>(1, hm.size()) * sizeof(MatDev));
    d_ent_ = DevBuf(pool, std::max<size_t>(1, he.size()) * sizeof(EntryDev));
    d_units_ = DevBuf(pool, std::max<size_t>(1, hu.size()) * sizeof(UnitDev));
    d_prefix_ = DevBuf(pool, (hu.size() + 1) * 8);
    if (!hu.empty()) copy_sync(d_units_.ptr, hu.data(), hu.size() * sizeof(UnitDev), hipMemcpyHostToDevice, s_);
    copy_sync(d_inst_.ptr, hi.data(), hi.size() * sizeof(InstDev), hipMemcpyHostToDevice, s_);
    if (!hm.empty())
        copy_sync(d_mats_.ptr, hm.data(), hm.size() * sizeof(MatDev), hipMemcpyHostToDevice, s_);
    if (!he.empty())
        copy_sync(d_ent_.ptr, he.data(), he.size() * sizeof(EntryDev), hipMemcpyHostToDevice, s_);
    if (opts_.count_traffic) {
        touched_bits_ = tbits;
        d_touched_ = DevBuf(pool, std::max<uint64_t>(8, (tbits + 31) / 32 * 4));
        d_touched_off_ = DevBuf(pool, toff.size() * 8);
        copy_sync(d_touched_off_.ptr, toff.data(), toff.size() * 8, hipMemcpyHostToDevice, s_);
    }
    dirty_ = false;
}

void Run::sort_appended() {
    SortArgs S{};
    S.inst = d_inst_.as<InstDev>();
    S.mats = d_mats_.as<MatDev>();
    S.ap_key = d_ap_key_.as<uint32_t>();
    S.ap_i = d_ap_i_.as<uint32_t>();
    S.ap_j = d_ap_j_.as<uint32_t>();
    S.ap_count = d_counters_.as<unsigned long long>();
    S.ap_cap = ap_cap_;
    S.rcnt = d_rcnt_.as<uint32_t>();
    S.ccnt = d_ccnt_.as<uint32_t>();
    S.rs = d_rs_.as<uint64_t>();
    S.cs = d_cs_.as<uint64_t>();
    S.rs_stage = d_rs_stage_.as<uint64_t>();
    S.cs_stage = d_cs_stage_.as<uint64_t>();
    S.halt = reinterpret_cast<uint32_t *>(d_counters_.as<unsigned long long>() + 3);
    hip_check(launch_sort(S, bucket_hi(), d_bsum_.as<uint32_t>(), ctx_->num_cu * 8, s_), "sort");
    // the appended pairs are consumed
    hip_check(launch_reset_appends(d_counters_.as<unsigned long long>(), S.halt, s_), "reset");
}

void Run::read_flags() {
    hip_check(hipMemcpyAsync(h_over_, d_inst_over_.ptr, (uint64_t)max_inst_ * 4, hipMemcpyDeviceToHost, s_),
              "D2H");
    hip_check(hipMemcpyAsync(h_counters_, d_counters_.ptr, 32, hipMemcpyDeviceToHost, s_), "D2H");
    hip_check(hipMemcpyAsync(h_stats_, d_slot_stats_.ptr, (uint64_t)max_inst_ * sizeof(SlotStats),
                             hipMemcpyDeviceToHost, s_),
              "D2H");
    hip_check(hipStreamSynchronize(s_), "sync");
}

// Δ := M for every instance: the naive variant (Algorithm 1 as printed,
// every pair takes part in every round), done before a round's sort.
void Run::extract_all_pairs() {
    hip_check(launch_fill_u64(d_counters_.as<unsigned long long>(), 1, 0, s_), "fill");
    // the pending pairs are dropped (every pair of M is new again): so are their counts
    hip_check(launch_zero_counts(d_rcnt_.as<uint32_t>(), d_ccnt_.as<uint32_t>(), bucket_hi() + 1,
                                 reinterpret_cast<uint32_t *>(d_counters_.as<unsigned long long>() + 3), s_),
              "zero counts");
    uint64_t total_pairs = 0;
    for (auto &ip : insts_) {
        DevBuf cnt(ctx_->pool.get(), std::max<uint32_t>(1, ip->n) * 4ull);
        DevBuf tot(ctx_->pool.get(), 8);
        hip_check(launch_fill_u64(tot.as<unsigned long long>(), 1, 0, s_), "fill");
        for (uint32_t x = 0; x < ip->low.nmat(); x++)
            hip_check(launch_row_count(ip->mats[x].R, ip->n, ip->S, cnt.as<uint32_t>(), tot.as<unsigned long long>(),
                                       s_),
                      "count");
        unsigned long long t = 0;
        copy_sync(&t, tot.ptr, 8, hipMemcpyDeviceToHost, s_);
        total_pairs += t;
    }
    ensure_capacity(total_pairs, false);
    for (auto &ip : insts_) {
        DevBuf dm(ctx_->pool.get(), ip->mats.size() * sizeof(MatDev));
        copy_sync(dm.ptr, ip->mats.data(), ip->mats.size() * sizeof(MatDev), hipMemcpyHostToDevice, s_);
        InstDev I{ip->n, ip->S, ip->bbase, 0};
        hip_check(launch_extract_all(dm.as<MatDev>(), I, ip->slot, ip->low.nmat(), d_ap_key_.as<uint32_t>(),
                                     d_ap_i_.as<uint32_t>(), d_ap_j_.as<uint32_t>(),
                                     d_counters_.as<unsigned long long>(), ap_cap_,
                                     d_inst_over_.as<uint32_t>() + ip->slot, d_rcnt_.as<uint32_t>(),
                                     d_ccnt_.as<uint32_t>(), s_),
                  "extract");
        hip_check(hipStreamSynchronize(s_), "sync");
    }
}

void Run::enqueue_product(bool timed, bool rerun) {
    unsigned long long *counters = d_counters_.as<unsigned long long>();
    uint32_t *halt = reinterpret_cast<uint32_t *>(counters + 3);
    if (!nunit_) return;
    PrepArgs P{};
    P.units = d_units_.as<UnitDev>();
    P.nunit = nunit_;
    P.rptr = d_rcnt_.as<uint32_t>();
    P.cptr = d_ccnt_.as<uint32_t>();
    P.item_prefix = d_prefix_.as<uint64_t>();
    P.work_counter0 = counters + 1;
    P.work_counter1 = counters + 4;
    P.halt = halt;
    P.chunk = opts_.chunk_pairs ? opts_.chunk_pairs : (ctx_->chunk_pairs_tuned ? ctx_->chunk_pairs_tuned : kChunkPairs);
    P.ap_cap = ap_cap_;
    if (!rerun) {
        // the prep reads the bucket starts of this round's new pairs; then
        // the counters are cleared and the product counts the next round's
        hip_check(launch_prep(P, s_), "prep");
        hip_check(launch_zero_counts(d_rcnt_.as<uint32_t>(), d_ccnt_.as<uint32_t>(), bucket_hi() + 1, halt, s_),
                  "zero counts");
    } else {
        hip_check(launch_fill_u64(counters + 1, 1, 0, s_), "fill");
        hip_check(launch_fill_u64(counters + 4, 1, 0, s_), "fill");
    }
    if (opts_.count_traffic && touched_bits_)
        hip_check(launch_fill_u32(d_touched_.as<uint32_t>(), (touched_bits_ + 31) / 32, 0, s_), "fill");
    ProductArgs A{};
    A.mats = d_mats_.as<MatDev>();
    A.units = d_units_.as<UnitDev>();
    A.item_prefix = d_prefix_.as<uint64_t>();
    A.rs = d_rs_.as<uint64_t>();
    A.cs = d_cs_.as<uint64_t>();
    A.ap_key = d_ap_key_.as<uint32_t>();
    A.ap_i = d_ap_i_.as<uint32_t>();
    A.ap_j = d_ap_j_.as<uint32_t>();
    A.ap_count = counters;
    A.ap_cap = ap_cap_;
    A.inst_overflow = d_inst_over_.as<uint32_t>();
    A.halt = halt;
    A.inst_new = d_inst_new_.as<unsigned long long>();
    A.touched = d_touched_.as<uint32_t>();
    A.touched_off = d_touched_off_.as<uint64_t>();
    A.algo_bytes = counters + 2;
    A.chunk = P.chunk;
    A.rcnt = d_rcnt_.as<uint32_t>();
    A.ccnt = d_ccnt_.as<uint32_t>();
    if (timed) hip_check(hipEventRecord(ev0_, s_), "event");
    // the row parts, then the column parts (a pair derived by both is then
    // reported once: by the row part)
    A.unit_lo = 0;
    A.unit_hi = unit_split_;
    A.work_counter = counters + 1;
    hip_check(launch_product(A, grid_, opts_.count_traffic != 0, s_), "product");
    A.unit_lo = unit_split_;
    A.unit_hi = nunit_;
    A.work_counter = counters + 4;
    hip_check(launch_product(A, grid_, opts_.count_traffic != 0, s_), "product");
    if (timed) hip_check(hipEventRecord(ev1_, s_), "event");
    product_launches_ += 2;
}

// End of a round: fold the new-pair counts into the per-instance statistics.
void Run::enqueue_round_end() {
    unsigned long long *counters = d_counters_.as<unsigned long long>();
    uint32_t *halt = reinterpret_cast<uint32_t *>(counters + 3);
    hip_check(launch_round_end(d_active_.as<uint32_t>(), d_inst_new_.as<unsigned long long>(),
                               d_slot_stats_.as<SlotStats>(), max_inst_, halt, s_),
              "round_end");
}

// One round without host synchronisation: sort the pending new pairs into
// dA / dB, run the product, fold the counts.  Every kernel skips its
// work once an overflow has set the halt flag.
void Run::enqueue_round(bool timed) {
    sort_appended();
    enqueue_product(timed);
    enqueue_round_end();
}

// After an overflow: the product of the overflowing round left M unchanged
// for the candidates it could not append; dA / dB of that round are still in
// rs / cs.  Grow the buffer (keeping [0, cap)), re-run that product.
void Run::recover() {
    unsigned long long *counters = d_counters_.as<unsigned long long>();
    uint32_t *halt = reinterpret_cast<uint32_t *>(counters + 3);
    for (int attempt = 0; (uint32_t)(h_counters_[3] & 0xFFFFFFFFu); attempt++) {
        if (attempt > 64) throw Error(CFLR_ENOMEM, "new-pair buffer keeps overflowing");
        reruns_++;
        const uint64_t asked = h_counters_[0];
        const uint64_t old_cap = ap_cap_;
        ensure_capacity(std::max<uint64_t>(2 * old_cap, asked + asked / 2), true);
        unsigned long long v = old_cap;
        copy_sync(counters, &v, 8, hipMemcpyHostToDevice, s_);
        hip_check(launch_fill_u32(halt, 1, 0, s_), "fill");
        hip_check(launch_fill_u32(d_inst_over_.as<uint32_t>(), max_inst_, 0, s_), "fill");
        enqueue_product(false, true);
        enqueue_round_end();
        read_flags();
    }
}

uint32_t Run::round() { return rounds(1); }

uint32_t Run::rounds(uint32_t R) {
    if (insts_.empty()) return 0;
    rebuild_tables();
    const bool eager = R <= 1 || !opts_.semi_naive || opts_.kernel_timing || opts_.count_traffic ||
                       s_ == nullptr;
    if (eager) {
        for (uint32_t r = 0; r < std::max<uint32_t>(1, R); r++) {
            if (!opts_.semi_naive) extract_all_pairs();
            enqueue_round(opts_.kernel_timing != 0);
            read_flags();
            if (opts_.kernel_timing && nunit_) {
                float ms = 0;
                hip_check(hipEventElapsedTime(&ms, ev0_, ev1_), "event");
                product_ms_ += ms;
            }
            if ((uint32_t)(h_counters_[3] & 0xFFFFFFFFu)) recover();
            if (log_) log_round();
            round_no_++;
        }
    } else {
        // capture R rounds once per table/buffer generation, then replay
        if (!graph_exec_ || graph_gen_ != generation_ || graph_rounds_ != R) {
            if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
            graph_exec_ = nullptr;
            hipGraph_t g = nullptr;
            hip_check(hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal), "capture");
            for (uint32_t r = 0; r < R; r++) enqueue_round(false);
            hip_check(hipStreamEndCapture(s_, &g), "capture");
            hip_check(hipGraphInstantiate(&graph_exec_, g, nullptr, nullptr, 0), "instantiate");
            (void)hipGraphDestroy(g);
            graph_gen_ = generation_;
            graph_rounds_ = R;
            product_launches_ -= R;  // counted below, per replay
        }
        hip_check(hipGraphLaunch(graph_exec_, s_), "graph launch");
        product_launches_ += nunit_ ? R : 0;
        read_flags();
        if ((uint32_t)(h_counters_[3] & 0xFFFFFFFFu)) recover();
        if (log_) log_round();
        round_no_ += R;
    }
    if (opts_.count_traffic) algo_bytes_ = h_counters_[2];
    uint32_t running = 0;
    for (auto &ip : insts_) {
        Instance &in = *ip;
        const SlotStats &st = h_stats_[in.slot];
        in.rounds = st.rounds;
        in.stats.new_pairs = st.new_total;
        in.stats.max_delta = st.max_delta;
        in.done = st.done != 0;
        if (!in.done) running++;
    }
    return running;
}

void Run::log_round() {
    uint64_t items = 0;
    if (nunit_) copy_sync(&items, d_prefix_.as<uint64_t>() + nunit_, 8, hipMemcpyDeviceToHost, s_);
    uint64_t fresh = 0;
    for (auto &ip : insts_) fresh += h_stats_[ip->slot].new_total;
    std::fprintf(stderr, "[cflr] round %u: instances %zu items %llu appended %llu derived-so-far %llu cap %llu reruns %u\n",
                 (unsigned)round_no_, insts_.size(), (unsigned long long)items, (unsigned long long)h_counters_[0],
                 (unsigned long long)fresh, (unsigned long long)ap_cap_, reruns_);
}

// ------------------------------------------------------------------ readout

void instance_counts(Instance &inst) {
    bool need = false;
    for (auto c : inst.counts) need |= c < 0;
    if (!need) return;
    if (inst.sp) {
        sparse_counts(inst);
        return;
    }
    cflr_ctx *ctx = inst.ctx;
    hipStream_t s = ctx->stream;
    const uint32_t U = (uint32_t)inst.low.user_names.size();
    DevBuf cnt(ctx->pool.get(), std::max<uint32_t>(1, inst.n) * 4ull);
    DevBuf tot(ctx->pool.get(), 8ull * U);
    hip_check(hipMemsetAsync(tot.ptr, 0, 8ull * U, s), "memset");
    for (uint32_t x = 0; x < U; x++)
        hip_check(launch_row_count(inst.mats[x].R, inst.n, inst.S, cnt.as<uint32_t>(),
                                   tot.as<unsigned long long>() + x, s),
                  "count");
    std::vector<unsigned long long> h(U);
    hip_check(hipMemcpyAsync(h.data(), tot.ptr, 8ull * U, hipMemcpyDeviceToHost, s), "D2H");
    hip_check(hipStreamSynchronize(s), "sync");
    uint64_t total = 0;
    for (uint32_t x = 0; x < U; x++) {
        inst.counts[x] = (int64_t)h[x];
        total += h[x];
    }
    inst.stats.total_pairs = total;
}

void instance_copy(Instance &inst, uint32_t nt, uint32_t *src, uint32_t *dst, uint64_t capacity,
                   bool on_device, uint64_t *written) {
    instance_counts(inst);
    const uint64_t count = (uint64_t)inst.counts[nt];
    if (capacity < count) throw Error(CFLR_EINVAL, "capacity smaller than the pair count");
    *written = count;
    if (!count) return;
    if (inst.sp) {
        sparse_copy(inst, nt, src, dst, count, on_device);
        return;
    }
    cflr_ctx *ctx = inst.ctx;
    hipStream_t s = ctx->stream;
    DevBuf cnt(ctx->pool.get(), (uint64_t)inst.n * 4);
    DevBuf off(ctx->pool.get(), (uint64_t)inst.n * 8);
    hip_check(launch_row_count(inst.mats[nt].R, inst.n, inst.S, cnt.as<uint32_t>(), nullptr, s), "count");
    if (on_device) {
        hip_check(launch_row_write(inst.mats[nt].R, inst.n, inst.S, cnt.as<uint32_t>(), off.as<uint64_t>(), src,
                                   dst, s),
                  "readout");
        hip_check(hipStreamSynchronize(s), "sync");
        return;
    }
    DevBuf dsrc(ctx->pool.get(), count * 4), ddst(ctx->pool.get(), count * 4);
    hip_check(launch_row_write(inst.mats[nt].R, inst.n, inst.S, cnt.as<uint32_t>(), off.as<uint64_t>(),
                               dsrc.as<uint32_t>(), ddst.as<uint32_t>(), s),
              "readout");
    hip_check(hipMemcpyAsync(src, dsrc.ptr, count * 4, hipMemcpyDeviceToHost, s), "D2H");
    hip_check(hipMemcpyAsync(dst, ddst.ptr, count * 4, hipMemcpyDeviceToHost, s), "D2H");
    hip_check(hipStreamSynchronize(s), "sync");
}

}  // namespace cflr

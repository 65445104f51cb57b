// sparse.cpp -- host side of the sparse storage engine (layout in sparse.h).
//
// The fixpoint of Algorithm 1 in its semi-naive form (Section 3, opt. 1):
//   seed      edges and eps rules insert the first pairs (the first round's
//             new pairs);
//   round r   the new pairs of round r-1 are added to the adjacency lists,
//             then every one of them meets the partner lists of the
//             productions that use its matrix; candidates are inserted into
//             the hash set, and the inserts that succeed are round r's new
//             pairs;
//   converge  a round that derives no pair ends the solve.
// Overflows (the pool of list entries, the new-pair buffer, the hash set)
// halt the round's remaining kernels; the host grows the structure and
// resumes or re-runs the step.  A re-run is exact: a pair already inserted
// is found again and not reported twice, and the pairs whose insert was
// taken back are inserted again.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "engine.h"
#include "sparse.h"

namespace cflr {

using sp::kNone;

namespace {

struct Plan {
    std::vector<sp::MatInfo> mats;
    std::vector<sp::Use> uses;
    std::vector<uint32_t> obs_ptr;
    std::vector<sp::Obs> obs;
    uint32_t nlayouts = 0;
    uint64_t mask_words = 0;
    uint32_t nrank0 = 0, nrank1 = 0;  // matrices with part 0 (part 1) uses
};

// Layouts, use tables and observers of a lowered grammar on n vertices.
// Row layouts: matrices in a b slot and the text's non-terminals (results
// are read out by rows); column layouts: matrices in an a slot.
Plan make_plan(const Lowered &low, uint32_t n) {
    Plan P;
    const uint32_t M = low.nmat(), U = (uint32_t)low.user_names.size();
    sp::MatInfo none{};
    none.row_layout = none.col_layout = kNone;
    none.rank0 = none.rank1 = kNone;
    P.mats.assign(M, none);
    for (uint32_t x = 0; x < M; x++)
        if (low.slot_b[x] || x < U) P.mats[x].row_layout = P.nlayouts++;
    for (uint32_t x = 0; x < M; x++)
        if (low.slot_a[x]) P.mats[x].col_layout = P.nlayouts++;
    std::vector<std::vector<sp::Use>> u0(M), u1(M);
    for (const auto &b : low.binary) {
        u0[b.a].push_back(sp::Use{b.c, P.mats[b.b].row_layout});
        u1[b.b].push_back(sp::Use{b.c, P.mats[b.a].col_layout});
    }
    std::vector<std::vector<sp::Obs>> ob(P.nlayouts);
    uint64_t mw = 0;
    for (uint32_t x = 0; x < M; x++) {
        sp::MatInfo &mi = P.mats[x];
        for (int part = 0; part < 2; part++) {
            const auto &list = part == 0 ? u0[x] : u1[x];
            const uint32_t first = (uint32_t)P.uses.size(), cnt = (uint32_t)list.size();
            const uint32_t words = (cnt + 63) / 64;
            for (uint32_t q = 0; q < cnt; q++) {
                if (list[q].layout == kNone) throw Error(CFLR_EDEVICE, "internal: production without a partner layout");
                P.uses.push_back(list[q]);
                ob[list[q].layout].push_back(sp::Obs{mw, words, q});
            }
            if (part == 0) {
                mi.use0 = first;
                mi.nuse0 = cnt;
                mi.w0 = words;
                mi.mask0 = mw;
                if (cnt) mi.rank0 = P.nrank0++;
            } else {
                mi.use1 = first;
                mi.nuse1 = cnt;
                mi.w1 = words;
                mi.mask1 = mw;
                if (cnt) mi.rank1 = P.nrank1++;
            }
            mw += (uint64_t)n * words;
        }
    }
    P.mask_words = mw;
    P.obs_ptr.assign(P.nlayouts + 1, 0);
    for (uint32_t L = 0; L < P.nlayouts; L++) {
        P.obs_ptr[L + 1] = P.obs_ptr[L] + (uint32_t)ob[L].size();
        for (auto &o : ob[L]) P.obs.push_back(o);
    }
    return P;
}

uint64_t pow2_at_least(uint64_t v) {
    uint64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

template <class T>
void upload(DevBuf &buf, DevPool *pool, const std::vector<T> &v, hipStream_t s) {
    buf = DevBuf(pool, std::max<size_t>(1, v.size()) * sizeof(T));
    if (!v.empty()) copy_sync(buf.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

// A new-pair buffer with its own count word.
struct Buf {
    DevBuf key, i, j, count;
    uint64_t cap = 0;
    sp::PairBuf dev() const {
        return sp::PairBuf{key.as<uint32_t>(), i.as<uint32_t>(), j.as<uint32_t>(),
                           count.as<unsigned long long>(), cap};
    }
};

void alloc_buf(Buf &b, DevPool *pool, uint64_t cap, hipStream_t s) {
    b.key = DevBuf(pool, cap * 4);
    b.i = DevBuf(pool, cap * 4);
    b.j = DevBuf(pool, cap * 4);
    if (!b.count.ptr) b.count = DevBuf(pool, 8);
    b.cap = cap;
    hip_check(sp::launch_fill_u64(b.count.as<unsigned long long>(), 1, 0, s), "fill");
}

// Grow a buffer to new_cap entries keeping [0, cap); its count becomes the
// old capacity (the entries there are pairs or holes).
void grow_buf(Buf &b, DevPool *pool, uint64_t new_cap, hipStream_t s) {
    DevBuf k(pool, new_cap * 4), i(pool, new_cap * 4), j(pool, new_cap * 4);
    hip_check(hipMemcpyAsync(k.ptr, b.key.ptr, b.cap * 4, hipMemcpyDeviceToDevice, s), "D2D");
    hip_check(hipMemcpyAsync(i.ptr, b.i.ptr, b.cap * 4, hipMemcpyDeviceToDevice, s), "D2D");
    hip_check(hipMemcpyAsync(j.ptr, b.j.ptr, b.cap * 4, hipMemcpyDeviceToDevice, s), "D2D");
    unsigned long long c = b.cap;
    hip_check(hipMemcpyAsync(b.count.ptr, &c, 8, hipMemcpyHostToDevice, s), "H2D");
    hip_check(hipStreamSynchronize(s), "sync");
    b.key = std::move(k);
    b.i = std::move(i);
    b.j = std::move(j);
    b.cap = new_cap;
}

}  // namespace

// ------------------------------------------------------------------- solve

void sparse_solve(cflr_ctx *ctx, const cflr_opts &o, Instance &inst, bool *timed_out) {
    *timed_out = false;
    hipStream_t s = ctx->stream;
    DevPool *pool = ctx->pool.get();
    const Lowered &low = inst.low;
    const uint32_t n = inst.n;
    if (n >= sp::kMaxVertices) throw Error(CFLR_EUNSUPPORTED, "sparse storage holds at most 2^24 - 1 vertices");
    if (low.nmat() >= sp::kMaxMatrices) throw Error(CFLR_EUNSUPPORTED, "grammar needs 65535 or more matrices");
    const bool log = std::getenv("CFLR_LOG") != nullptr;
    Plan P = make_plan(low, n);

    auto store = std::make_shared<SparseStore>();
    store->hold = CtxRef(ctx);
    store->ctx = ctx;
    store->n = n;
    store->nlayouts = P.nlayouts;
    store->row_layout.resize(low.nmat());
    for (uint32_t x = 0; x < low.nmat(); x++) store->row_layout[x] = P.mats[x].row_layout;

    DevBuf d_mats, d_uses, d_obs_ptr, d_obs;
    upload(d_mats, pool, P.mats, s);
    upload(d_uses, pool, P.uses, s);
    upload(d_obs_ptr, pool, P.obs_ptr, s);
    upload(d_obs, pool, P.obs, s);
    const uint64_t cells = (uint64_t)P.nlayouts * n;
    store->dir = DevBuf(pool, std::max<uint64_t>(1, cells) * sizeof(sp::Dir));
    DevBuf d_cur(pool, std::max<uint64_t>(1, cells) * 4);
    DevBuf d_mask(pool, std::max<uint64_t>(1, P.mask_words) * 8);
    DevBuf d_ctl(pool, sp::kCtlWords * 8);
    if (cells) {
        hip_check(hipMemsetAsync(store->dir.ptr, 0, cells * sizeof(sp::Dir), s), "memset");
        hip_check(hipMemsetAsync(d_cur.ptr, 0, cells * 4, s), "memset");
    }
    if (P.mask_words) hip_check(hipMemsetAsync(d_mask.ptr, 0, P.mask_words * 8, s), "memset");
    hip_check(hipMemsetAsync(d_ctl.ptr, 0, sp::kCtlWords * 8, s), "memset");

    const uint32_t grid = std::max<uint32_t>(1, ctx->num_cu * 8);
    uint32_t waves = o.grid_waves ? o.grid_waves : ctx->grid_waves_tuned;
    if (!waves) waves = ctx->num_cu * 32;
    const uint64_t slack = 2ull * waves * 64;  // keys a halted round may insert and take back

    // new-pair buffers; the first holds the seeds (their count is bounded).
    // Capacities start at what earlier solves on this context grew to
    // (bounded by the size of this input), or at opts.delta_capacity.
    const uint64_t seeds_max = inst.max_seeds;
    const uint64_t scale = std::max<uint64_t>(1ull << 16, 4096 * seeds_max);
    uint64_t cap_out = o.delta_capacity ? std::max<uint64_t>(64, o.delta_capacity)
                                        : std::max<uint64_t>(1ull << 16, std::min(ctx->sparse_delta_hint, scale));
    const uint64_t seed_slack = 2ull * 4 * sp::kSeedBlocks * sp::kChunk;
    Buf A, B;
    alloc_buf(A, pool, std::max(cap_out, seeds_max + seed_slack), s);
    alloc_buf(B, pool, cap_out, s);

    // hash set: at most 70 % full, counting what the next round may add
    uint64_t hash_keys = 0;       // pairs in the table
    uint64_t tombs_resident = 0;  // tombstones in the table (a rehash drops them)
    uint64_t slots = 0;
    DevBuf hash;
    auto hash_need = [&](uint64_t extra) {
        return pow2_at_least((hash_keys + tombs_resident + extra + slack) * 10 / 7 + 1);
    };
    sp::State S{};
    auto rehash_to = [&](uint64_t new_slots) {
        if (new_slots & (new_slots - 1)) throw Error(CFLR_EDEVICE, "internal: hash slots not a power of two");
        DevBuf nh(pool, new_slots * 8);
        hip_check(sp::launch_fill_u64(nh.as<unsigned long long>(), new_slots, sp::kEmpty, s), "fill");
        if (slots) {
            S.hash = nh.as<unsigned long long>();
            S.hash_mask = new_slots - 1;
            hip_check(sp::launch_rehash(S, hash.as<unsigned long long>(), slots, s), "rehash");
        }
        hash = std::move(nh);
        slots = new_slots;
        S.hash = hash.as<unsigned long long>();
        S.hash_mask = slots - 1;
        tombs_resident = 0;
        hip_check(sp::launch_fill_u64(S.ctl + sp::kCtlTomb, 1, 0, s), "fill");
    };

    // the pool of list entries
    uint64_t pool_cap = std::max<uint64_t>(1ull << 20, 4 * seeds_max);
    if (!o.delta_capacity) pool_cap = std::max(pool_cap, std::min(ctx->sparse_pool_hint, 16 * scale));
    DevBuf d_pool(pool, pool_cap * 4);
    DevBuf d_touched, d_moves;
    uint64_t touched_cap = 0;

    // the grouped product: new pairs sorted by (matrix, key); buckets whose
    // products reach `threshold` (n / 2 by default: below that the per-item
    // cost of the bit set outweighs the hash probes it saves, measured on
    // the 200,000-vertex points-to graph) are expanded into an LDS bit set.
    // Off when the bucket space or the bit set is too large.
    sp::KeySort K{};
    K.nb0 = (uint64_t)P.nrank0 * n;
    K.nb = K.nb0 + (uint64_t)P.nrank1 * n;
    const bool grouped = K.nb > 0 && K.nb < (1ull << 30) && sp::heavy_lds_bytes(n) <= sp::kHeavyMaxLds &&
                         std::getenv("CFLR_SPARSE_UNGROUPED") == nullptr;
    K.threshold = std::max<uint64_t>(1, n / 2);
    if (const char *h = std::getenv("CFLR_SPARSE_HEAVY")) K.threshold = std::max<uint64_t>(1, std::strtoull(h, nullptr, 10));
    K.big_entry = 0x7FFFFFFFu;
    if (const char *h = std::getenv("CFLR_SPARSE_BIG")) K.big_entry = (uint32_t)std::strtoul(h, nullptr, 10);
    DevBuf k_start, k_work, k_bsum, k_entry, k_heavy, k_ework;
    if (grouped) {
        k_start = DevBuf(pool, (K.nb + 1) * 4);
        k_work = DevBuf(pool, K.nb * 8);
        k_bsum = DevBuf(pool, sp::key_sort_scan_blocks(K.nb) * 4);
        K.start = k_start.as<uint32_t>();
        K.work = k_work.as<unsigned long long>();
        K.bsum = k_bsum.as<uint32_t>();
    }

    S.n = n;
    S.nlayouts = P.nlayouts;
    S.mats = d_mats.as<sp::MatInfo>();
    S.uses = d_uses.as<sp::Use>();
    S.obs_ptr = d_obs_ptr.as<uint32_t>();
    S.obs = d_obs.as<sp::Obs>();
    S.dir = store->dir.as<sp::Dir>();
    S.cur = d_cur.as<uint32_t>();
    S.mask = d_mask.as<uint64_t>();
    S.pool = d_pool.as<uint32_t>();
    S.pool_cap = pool_cap;
    S.ctl = d_ctl.as<unsigned long long>();
    rehash_to(pow2_at_least(
        std::max(hash_need(seeds_max), o.delta_capacity ? 0 : std::min(ctx->sparse_slots_hint, 16 * scale))));

    unsigned long long *h_ctl = nullptr;
    hip_check(hipHostMalloc((void **)&h_ctl, (sp::kCtlWords + 2) * 8, 0), "hipHostMalloc");
    struct PinFree {
        unsigned long long *p;
        ~PinFree() { (void)hipHostFree(p); }
    } pin_guard{h_ctl};
    auto read_ctl = [&](const Buf *out) {
        hip_check(hipMemcpyAsync(h_ctl, d_ctl.ptr, sp::kCtlWords * 8, hipMemcpyDeviceToHost, s), "D2H");
        if (out) hip_check(hipMemcpyAsync(h_ctl + sp::kCtlWords, out->count.ptr, 8, hipMemcpyDeviceToHost, s), "D2H");
        hip_check(hipStreamSynchronize(s), "sync");
    };
    auto clear_flags = [&]() {
        // halt, overflow flags; keep the pool top and the tombstone count
        const int words[] = {sp::kCtlHalt,     sp::kCtlPoolOver,   sp::kCtlBufOver,         sp::kCtlHashFull,
                             sp::kCtlTasks,    sp::kCtlProducts,   sp::kCtlHeavyTasks,      sp::kCtlHeavyProducts,
                             sp::kCtlHeavyCand};
        for (int w : words) hip_check(sp::launch_fill_u64(S.ctl + w, 1, 0, s), "fill");
    };

    // ---- seeds (a re-run after an overflow inserts only what is missing)
    hip_check(sp::launch_round_start(S, s), "round start");
    for (int attempt = 0;; attempt++) {
        hip_check(sp::launch_seed(S, inst.graph->src.as<uint32_t>(), inst.graph->dst.as<uint32_t>(),
                                  inst.graph->lab.as<uint32_t>(), inst.graph->m, inst.lm_ptr.as<uint32_t>(),
                                  inst.lm_mat.as<uint32_t>(), inst.eps_mat.as<uint32_t>(), inst.n_eps, A.dev(), s),
                  "seed");
        read_ctl(&A);
        if (!h_ctl[sp::kCtlHalt]) break;
        if (attempt > 64) throw Error(CFLR_ENOMEM, "seeding keeps overflowing");
        if (h_ctl[sp::kCtlBufOver]) {
            const uint64_t asked = h_ctl[sp::kCtlWords];
            grow_buf(A, pool, std::max<uint64_t>(2 * A.cap, asked + asked / 2), s);
        }
        const uint64_t resident = h_ctl[sp::kCtlNew] + h_ctl[sp::kCtlTomb];
        uint64_t want = pow2_at_least((resident + seeds_max + slack) * 10 / 7 + 1);
        if (h_ctl[sp::kCtlHashFull]) want = std::max(want, 2 * slots);
        if (want > slots) rehash_to(want);
        clear_flags();
    }
    uint64_t pending = h_ctl[sp::kCtlNew];
    inst.stats.seed_pairs = pending;
    hash_keys += pending;
    tombs_resident += h_ctl[sp::kCtlTomb];
    hip_check(sp::launch_fill_u64(S.ctl + sp::kCtlTomb, 1, 0, s), "fill");

    Buf *in = &A, *out = &B;
    uint32_t rounds = 0;
    uint64_t new_total = 0, max_delta = 0;
    double product_ms = 0;
    uint64_t launches = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (o.kernel_timing) {
        hip_check(hipEventCreate(&ev0), "event");
        hip_check(hipEventCreate(&ev1), "event");
    }
    while (pending) {
        if (o.max_rounds && rounds >= o.max_rounds) {
            *timed_out = true;
            break;
        }
        rounds++;
        // room for this round: hash load, touched lists, the output buffer
        const uint64_t want_slots = hash_need(out->cap);
        if (want_slots > slots) rehash_to(want_slots);
        if (touched_cap < 2 * in->cap) {
            touched_cap = 2 * in->cap;
            d_touched = DevBuf(pool, touched_cap * 8);
            d_moves = DevBuf(pool, std::max<uint64_t>(1, touched_cap / 4) * 24);
        }
        S.touched = d_touched.as<uint64_t>();
        S.touched_cap = touched_cap;
        S.moves = d_moves.as<uint64_t>();
        S.moves_cap = std::max<uint64_t>(1, touched_cap / 4);
        hip_check(sp::launch_fill_u64(out->count.as<unsigned long long>(), 1, 0, s), "fill");
        hip_check(sp::launch_round_start(S, s), "round start");

        // integrate the pending pairs into the lists
        hip_check(sp::launch_integrate(S, in->dev(), false, grid, s), "integrate");
        read_ctl(nullptr);
        while (h_ctl[sp::kCtlHalt]) {
            if (h_ctl[sp::kCtlTouchedOver]) throw Error(CFLR_EDEVICE, "internal: touched-list array too small");
            if (!h_ctl[sp::kCtlPoolOver]) throw Error(CFLR_EDEVICE, "internal: integration halted");
            const uint64_t top = h_ctl[sp::kCtlPoolTop], need = top + h_ctl[sp::kCtlAlloc];
            const uint64_t ncap = std::max<uint64_t>(2 * pool_cap, need + need / 2);
            DevBuf np(pool, ncap * 4);
            hip_check(hipMemcpyAsync(np.ptr, d_pool.ptr, top * 4, hipMemcpyDeviceToDevice, s), "D2D");
            hip_check(hipStreamSynchronize(s), "sync");
            d_pool = std::move(np);
            pool_cap = ncap;
            S.pool = d_pool.as<uint32_t>();
            S.pool_cap = pool_cap;
            if (log) std::fprintf(stderr, "[cflr] sparse: pool grown to %llu entries\n", (unsigned long long)ncap);
            clear_flags();
            hip_check(sp::launch_integrate(S, in->dev(), true, grid, s), "integrate");
            read_ctl(nullptr);
        }

        // the product
        if (grouped) {
            if (K.entry_cap < 2 * in->cap) {
                if (2 * in->cap >= (1ull << 32)) throw Error(CFLR_ENOMEM, "more than 2^31 new pairs in one round");
                K.entry_cap = K.heavy_cap = 2 * in->cap;
                k_entry = DevBuf(pool, K.entry_cap * 8);
                k_heavy = DevBuf(pool, K.heavy_cap * 4);
                k_ework = DevBuf(pool, K.entry_cap * 4);
                K.entry = k_entry.as<uint64_t>();
                K.heavy = k_heavy.as<uint32_t>();
                K.ework = k_ework.as<uint32_t>();
            }
            hip_check(sp::launch_key_sort(S, in->dev(), K, s), "key sort");
        }
        auto product = [&]() {
            if (grouped) hip_check(sp::launch_grouped_product(S, K, out->dev(), waves, s), "product");
            else hip_check(sp::launch_product(S, in->dev(), out->dev(), waves, s), "product");
        };
        hip_check(sp::launch_fill_u64(S.ctl + sp::kCtlNew, 1, 0, s), "fill");
        hip_check(sp::launch_fill_u64(S.ctl + sp::kCtlProducts, 1, 0, s), "fill");
        hip_check(sp::launch_fill_u64(S.ctl + sp::kCtlHeavyProducts, 2, 0, s), "fill");
        if (ev0) hip_check(hipEventRecord(ev0, s), "event");
        product();
        if (ev1) hip_check(hipEventRecord(ev1, s), "event");
        launches++;
        read_ctl(out);
        if (ev1) {
            float ms = 0;
            hip_check(hipEventElapsedTime(&ms, ev0, ev1), "event");
            product_ms += ms;
        }
        for (int attempt = 0; h_ctl[sp::kCtlHalt]; attempt++) {
            if (attempt > 64) throw Error(CFLR_ENOMEM, "new-pair buffer or hash set keeps overflowing");
            inst.stats.reruns++;
            if (h_ctl[sp::kCtlBufOver]) {
                const uint64_t asked = h_ctl[sp::kCtlWords];
                const uint64_t ncap = std::max<uint64_t>(2 * out->cap, asked + asked / 2);
                if (ncap > (1ull << 34)) throw Error(CFLR_ENOMEM, "new-pair buffer beyond 2^34 pairs");
                grow_buf(*out, pool, ncap, s);
            }
            // the table holds the pairs appended so far this round and the
            // tombstones of the halted run: room for what the re-run may add
            const uint64_t resident = hash_keys + h_ctl[sp::kCtlNew] + tombs_resident + h_ctl[sp::kCtlTomb];
            uint64_t want = pow2_at_least((resident + out->cap + slack) * 10 / 7 + 1);
            if (h_ctl[sp::kCtlHashFull]) want = std::max(want, 2 * slots);
            if (want > slots) rehash_to(want);  // drops the tombstones
            if (log)
                std::fprintf(stderr, "[cflr] sparse: round %u re-run (buffer %llu, slots %llu)\n", rounds,
                             (unsigned long long)out->cap, (unsigned long long)slots);
            clear_flags();
            if (ev0) hip_check(hipEventRecord(ev0, s), "event");
            product();
            if (ev1) hip_check(hipEventRecord(ev1, s), "event");
            launches++;
            read_ctl(out);
            if (ev1) {
                float ms = 0;
                hip_check(hipEventElapsedTime(&ms, ev0, ev1), "event");
                product_ms += ms;
            }
        }
        // kCtlNew counts every pair appended this round, over re-runs too
        const uint64_t fresh = h_ctl[sp::kCtlNew];
        new_total += fresh;
        hash_keys += fresh;
        tombs_resident += h_ctl[sp::kCtlTomb];
        hip_check(sp::launch_fill_u64(S.ctl + sp::kCtlTomb, 1, 0, s), "fill");
        max_delta = std::max(max_delta, fresh);
        if (log)
            std::fprintf(stderr,
                         "[cflr] sparse round %u: in %llu new %llu products %llu heavy items %llu products %llu "
                         "candidates %llu pool %llu/%llu slots %llu\n",
                         rounds, (unsigned long long)pending, (unsigned long long)fresh,
                         (unsigned long long)h_ctl[sp::kCtlProducts], (unsigned long long)h_ctl[sp::kCtlHeavy],
                         (unsigned long long)h_ctl[sp::kCtlHeavyProducts], (unsigned long long)h_ctl[sp::kCtlHeavyCand],
                         (unsigned long long)h_ctl[sp::kCtlPoolTop], (unsigned long long)pool_cap,
                         (unsigned long long)slots);
        pending = fresh;
        std::swap(in, out);
    }
    if (!pending && !*timed_out) rounds++;  // the round that derived nothing (counted as the dense engine does)
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    inst.rounds = rounds;
    inst.done = !*timed_out;
    inst.stats.rounds = rounds;
    inst.stats.new_pairs = new_total;
    inst.stats.max_delta = max_delta;
    inst.stats.product_ms = product_ms;
    inst.stats.product_launches = launches;
    ctx->sparse_delta_hint = std::max({ctx->sparse_delta_hint, A.cap, B.cap});
    ctx->sparse_pool_hint = std::max(ctx->sparse_pool_hint, pool_cap);
    ctx->sparse_slots_hint = std::max(ctx->sparse_slots_hint, slots);
    store->pool = std::move(d_pool);
    inst.stats.device_bytes = store->dir.bytes + store->pool.bytes;
    inst.sp = store;
}

// ------------------------------------------------------------------ readout

void sparse_counts(Instance &inst) {
    SparseStore &st = *inst.sp;
    cflr_ctx *ctx = inst.ctx;
    hipStream_t s = ctx->stream;
    const uint32_t U = (uint32_t)inst.low.user_names.size();
    DevBuf tot(ctx->pool.get(), 8ull * std::max<uint32_t>(1, U));
    hip_check(hipMemsetAsync(tot.ptr, 0, 8ull * std::max<uint32_t>(1, U), s), "memset");
    for (uint32_t x = 0; x < U; x++)
        hip_check(sp::launch_layout_count(st.dir.as<sp::Dir>() + (uint64_t)st.row_layout[x] * st.n, st.n,
                                          tot.as<unsigned long long>() + x, s),
                  "count");
    std::vector<unsigned long long> h(std::max<uint32_t>(1, U));
    hip_check(hipMemcpyAsync(h.data(), tot.ptr, 8ull * std::max<uint32_t>(1, U), hipMemcpyDeviceToHost, s), "D2H");
    hip_check(hipStreamSynchronize(s), "sync");
    uint64_t total = 0;
    for (uint32_t x = 0; x < U; x++) {
        inst.counts[x] = (int64_t)h[x];
        total += h[x];
    }
    inst.stats.total_pairs = total;
}

void sparse_copy(Instance &inst, uint32_t nt, uint32_t *src, uint32_t *dst, uint64_t count, bool on_device) {
    SparseStore &st = *inst.sp;
    cflr_ctx *ctx = inst.ctx;
    hipStream_t s = ctx->stream;
    DevPool *pool = ctx->pool.get();
    const uint32_t n = st.n;
    const uint32_t sort_grid = std::max<uint32_t>(1, std::min<uint32_t>(ctx->num_cu * 4, n));
    const uint64_t nw = ((uint64_t)n + 63) / 64;
    DevBuf off(pool, (uint64_t)n * 8), bm(pool, std::max<uint64_t>(1, (uint64_t)sort_grid * nw) * 8);
    hip_check(hipMemsetAsync(bm.ptr, 0, (uint64_t)sort_grid * nw * 8, s), "memset");
    const sp::Dir *dir = st.dir.as<sp::Dir>() + (uint64_t)st.row_layout[nt] * n;
    if (on_device) {
        hip_check(sp::launch_layout_write(dir, st.pool.as<uint32_t>(), n, off.as<uint64_t>(), bm.as<uint64_t>(),
                                          sort_grid, src, dst, s),
                  "readout");
        hip_check(hipStreamSynchronize(s), "sync");
        return;
    }
    DevBuf dsrc(pool, count * 4), ddst(pool, count * 4);
    hip_check(sp::launch_layout_write(dir, st.pool.as<uint32_t>(), n, off.as<uint64_t>(), bm.as<uint64_t>(), sort_grid,
                                      dsrc.as<uint32_t>(), ddst.as<uint32_t>(), s),
              "readout");
    hip_check(hipMemcpyAsync(src, dsrc.ptr, count * 4, hipMemcpyDeviceToHost, s), "D2H");
    hip_check(hipMemcpyAsync(dst, ddst.ptr, count * 4, hipMemcpyDeviceToHost, s), "D2H");
    hip_check(hipStreamSynchronize(s), "sync");
}

}  // namespace cflr

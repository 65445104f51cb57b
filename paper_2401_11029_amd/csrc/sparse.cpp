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
//
// Device memory comes from the context's caching pool, or -- for
// cflr_solve_noalloc, whose callers cannot allocate -- from the file-scope
// array `scratch` below, carved once per call; there every structure has a
// fixed size and an overflow ends the solve with CFLR_ENOMEM.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

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
    // per matrix: kNone, or the mirror whose row layout holds its pairs
    // transposed (a text's non-terminal that no kept production reads by
    // rows; its readout transposes the mirror's rows)
    std::vector<uint32_t> readout_mirror;
    std::vector<uint8_t> kept_head;  // per matrix: head of a production with uses
};

// The mirror of a grammar, when it has one.  Graphs of the paper's
// analyses hold every edge twice: (u, t, v) and its reverse (v, t_bar, u).
// If an involution s of the matrices maps every production c -> a b to a
// production s(c) -> s(b) s(a), every x -> t to s(x) -> t' (t' the reverse
// label of t) and keeps eps rules, and the seeds are their own mirror image
// ((x, i, j) seeded iff (s(x), j, i) is), then every round of the
// semi-naive fixpoint (Section 3, opt. 1) derives a mirror-closed set: by
// induction, s(c)'s candidates from s(b) s(a) are the transposes of c's
// from a b, with the same midpoints.  Only one production of each mirror
// pair then needs its product; the other's new pairs are the transposes.
// Labels pair by name: t and t_bar; a terminal without a partner is its
// own reverse.  s is found by refining candidate sets (a greatest fixpoint
// over the production structure), then checked exactly; mat[x] = s(x),
// rule[q] = the index of q's mirror production.
bool find_mirror(const Lowered &low, std::vector<uint32_t> *mat, std::vector<uint32_t> *rule) {
    const uint32_t M = low.nmat(), T = (uint32_t)low.terminals.size();
    if (!M || M > 8192 || low.binary.empty()) return false;
    std::map<std::string, uint32_t> tid;
    for (uint32_t t = 0; t < T; t++) tid[low.terminals[t]] = t;
    std::vector<uint32_t> tau(T);
    for (uint32_t t = 0; t < T; t++) tau[t] = t;
    // t_bar pairs with t, and an indexed t_bar_k with t_k
    const std::string bar = "_bar";
    for (uint32_t t = 0; t < T; t++) {
        const std::string &nm = low.terminals[t];
        for (size_t at = nm.find(bar); at != std::string::npos && at > 0; at = nm.find(bar, at + 1)) {
            const size_t end = at + bar.size();
            if (end != nm.size() && nm[end] != '_') continue;
            auto it = tid.find(nm.substr(0, at) + nm.substr(end));
            if (it != tid.end() && it->second != t) {
                tau[t] = it->second;
                tau[it->second] = t;
                break;
            }
        }
    }
    std::vector<uint8_t> eps(M, 0);
    for (uint32_t x : low.eps) eps[x] = 1;
    std::vector<std::vector<uint32_t>> terms(M), rterms(M);
    for (auto &tm : low.term) {
        terms[tm.second].push_back(tm.first);
        rterms[tm.second].push_back(tau[tm.first]);
    }
    for (uint32_t x = 0; x < M; x++) {
        std::sort(terms[x].begin(), terms[x].end());
        std::sort(rterms[x].begin(), rterms[x].end());
    }
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> bins(M);
    for (auto &b : low.binary) bins[b.c].push_back({b.a, b.b});
    // cand[x * M + y]: y may be s(x)
    std::vector<uint8_t> cand((size_t)M * M, 0);
    for (uint32_t x = 0; x < M; x++)
        for (uint32_t y = 0; y < M; y++)
            cand[(size_t)x * M + y] = eps[x] == eps[y] && rterms[x] == terms[y] && bins[x].size() == bins[y].size();
    for (bool changed = true; changed;) {
        changed = false;
        for (uint32_t x = 0; x < M; x++)
            for (uint32_t y = 0; y < M; y++) {
                if (!cand[(size_t)x * M + y]) continue;
                bool ok = cand[(size_t)y * M + x];
                for (size_t p = 0; ok && p < bins[x].size(); p++) {
                    const uint32_t a = bins[x][p].first, b = bins[x][p].second;
                    bool found = false;
                    for (auto &q : bins[y])
                        if (cand[(size_t)b * M + q.first] && cand[(size_t)a * M + q.second]) {
                            found = true;
                            break;
                        }
                    ok = found;
                }
                if (!ok) {
                    cand[(size_t)x * M + y] = 0;
                    changed = true;
                }
            }
    }
    // pick s from the candidates (first preferring another matrix, then x
    // itself) and check it exactly against the productions
    std::map<std::tuple<uint32_t, uint32_t, uint32_t>, uint32_t> prod;
    for (uint32_t q = 0; q < (uint32_t)low.binary.size(); q++) {
        const auto &b = low.binary[q];
        prod[std::make_tuple(b.c, b.a, b.b)] = q;
    }
    std::vector<uint32_t> s;
    auto attempt = [&](bool prefer_self) {
        s.assign(M, kNone);
        for (uint32_t x = 0; x < M; x++) {
            if (s[x] != kNone) continue;
            uint32_t pick = prefer_self && cand[(size_t)x * M + x] ? x : kNone;
            for (uint32_t y = 0; pick == kNone && y < M; y++)
                if (y != x && cand[(size_t)x * M + y] && s[y] == kNone) pick = y;
            if (pick == kNone && cand[(size_t)x * M + x]) pick = x;
            if (pick == kNone) return false;
            s[x] = pick;
            s[pick] = x;
        }
        rule->assign(low.binary.size(), kNone);
        for (uint32_t q = 0; q < (uint32_t)low.binary.size(); q++) {
            const auto &b = low.binary[q];
            auto it = prod.find(std::make_tuple(s[b.c], s[b.b], s[b.a]));
            if (it == prod.end()) return false;
            (*rule)[q] = it->second;
        }
        for (uint32_t x = 0; x < M; x++)
            if (s[s[x]] != x || eps[x] != eps[s[x]] || rterms[x] != terms[s[x]]) return false;
        return true;
    };
    if (!attempt(false) && !attempt(true)) return false;
    bool any = false;
    for (uint32_t q = 0; q < (uint32_t)rule->size(); q++) any = any || (*rule)[q] != q;
    if (!any) return false;  // nothing to save
    *mat = std::move(s);
    return true;
}

// Layouts, use tables and observers of a lowered grammar on n vertices.
// Row layouts: matrices in a b slot and the text's non-terminals (results
// are read out by rows); column layouts: matrices in an a slot.  Under a
// mirror plan (rule_mirror and mat_mirror non-empty) only one production of
// each mirror pair -- the one with the lower index -- gets uses, and only
// its operands' layouts are kept; x's column layout is then the row layout
// of its mirror s(x) (column j of x lists the i with x(i, j), which row j of
// s(x) lists), filled by s(x)'s pairs only.  With drop_readout, a text's
// non-terminal whose rows only the readout needs keeps none when its mirror
// has row lists: its pairs are read out as the mirror's, transposed.
Plan make_plan(const Lowered &low, uint32_t n, const std::vector<uint32_t> &rule_mirror,
               const std::vector<uint32_t> &mat_mirror, bool drop_readout) {
    Plan P;
    const uint32_t M = low.nmat(), U = (uint32_t)low.user_names.size();
    const uint32_t B = (uint32_t)low.binary.size();
    std::vector<uint8_t> keep(B, 1), slot_a(M, 0), slot_b(M, 0);
    for (uint32_t q = 0; q < B; q++) {
        if (!rule_mirror.empty() && rule_mirror[q] < q) keep[q] = 0;
        if (keep[q]) {
            slot_a[low.binary[q].a] = 1;
            slot_b[low.binary[q].b] = 1;
        }
    }
    sp::MatInfo none{};
    none.row_layout = none.col_layout = none.app_row = none.app_col = kNone;
    none.rank0 = none.rank1 = kNone;
    P.mats.assign(M, none);
    const bool alias = !mat_mirror.empty();
    P.readout_mirror.assign(M, kNone);
    std::vector<uint8_t> need_row(M, 0), head(M, 0);
    for (uint32_t q = 0; q < B; q++)
        if (keep[q]) head[low.binary[q].c] = 1;
    P.kept_head = head;
    for (uint32_t x = 0; x < M; x++) {
        if (slot_b[x] || (x < U && head[x])) need_row[x] = 1;  // read as a partner, or the head's own rows
        if (alias && slot_a[x] && mat_mirror[x] != x) need_row[mat_mirror[x]] = 1;
    }
    for (uint32_t x = 0; x < U; x++) {
        if (need_row[x]) continue;
        // rows only for the readout
        const uint32_t y = alias ? mat_mirror[x] : kNone;
        if (drop_readout && y != kNone && y != x && need_row[y]) {  // the mirror keeps rows: read x from them
            P.readout_mirror[x] = y;
            continue;
        }
        need_row[x] = 1;
    }
    for (uint32_t x = 0; x < M; x++)
        if (need_row[x]) P.mats[x].row_layout = P.mats[x].app_row = P.nlayouts++;
    for (uint32_t x = 0; x < M; x++) {
        if (!slot_a[x]) continue;
        if (alias && mat_mirror[x] != x) {
            P.mats[x].col_layout = P.mats[mat_mirror[x]].row_layout;  // a view: x appends nothing to it
        } else {
            P.mats[x].col_layout = P.mats[x].app_col = P.nlayouts++;
        }
    }
    std::vector<std::vector<sp::Use>> u0(M), u1(M);
    for (uint32_t q = 0; q < B; q++) {
        if (!keep[q]) continue;
        const auto &b = low.binary[q];
        u0[b.a].push_back(sp::Use{b.c, P.mats[b.b].row_layout, P.mats[b.c].row_layout, q});
        u1[b.b].push_back(sp::Use{b.c, P.mats[b.a].col_layout, P.mats[b.c].col_layout, q});
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

uint64_t pow2_at_most(uint64_t v) {
    uint64_t p = 1;
    while (2 * p <= v) p <<= 1;
    return p;
}

// Device memory of the engine: a block of the context's caching pool, or a
// piece of a fixed region (then `buf` is empty and nothing is freed).
struct Mem {
    DevBuf buf;
    void *ptr = nullptr;
    uint64_t bytes = 0;
    template <class T>
    T *as() const {
        return static_cast<T *>(ptr);
    }
};

class Alloc {
   public:
    explicit Alloc(DevPool *pool) : pool_(pool) {}
    Alloc(void *base, uint64_t cap) : base_(static_cast<char *>(base)), cap_(cap) {}
    bool fixed() const { return pool_ == nullptr; }
    Mem get(uint64_t bytes, const char *what) {
        Mem m;
        bytes = std::max<uint64_t>(1, bytes);
        if (pool_) {
            m.buf = DevBuf(pool_, bytes);
            m.ptr = m.buf.ptr;
            m.bytes = bytes;
            return m;
        }
        const uint64_t at = (top_ + 255) / 256 * 256;
        if (at > cap_ || bytes > cap_ - at)
            throw Error(CFLR_ENOMEM, std::string("input too large for the no-alloc scratch (") + what + " needs " +
                                         std::to_string(bytes) + " more bytes of " + std::to_string(cap_) + ")");
        m.ptr = base_ + at;
        m.bytes = bytes;
        top_ = at + bytes;
        return m;
    }
    // bytes of the fixed region not handed out yet
    uint64_t left() const {
        const uint64_t at = (top_ + 255) / 256 * 256;
        return at < cap_ ? cap_ - at : 0;
    }
    uint64_t mark() const { return top_; }
    void release_to(uint64_t mark) { top_ = mark; }

   private:
    DevPool *pool_ = nullptr;
    char *base_ = nullptr;
    uint64_t cap_ = 0, top_ = 0;
};

template <class T>
Mem upload(Alloc &A, const std::vector<T> &v, hipStream_t s, const char *what) {
    Mem m = A.get(std::max<size_t>(1, v.size()) * sizeof(T), what);
    if (!v.empty()) copy_sync(m.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
    return m;
}

// A new-pair buffer with its own count word.
struct Buf {
    Mem key, i, j, count;
    uint64_t cap = 0;
    sp::PairBuf dev() const {
        return sp::PairBuf{key.as<uint32_t>(), i.as<uint32_t>(), j.as<uint32_t>(),
                           count.as<unsigned long long>(), cap};
    }
};

void alloc_buf(Buf &b, Alloc &A, uint64_t cap, hipStream_t s) {
    b.key = A.get(cap * 4, "a new-pair buffer");
    b.i = A.get(cap * 4, "a new-pair buffer");
    b.j = A.get(cap * 4, "a new-pair buffer");
    if (!b.count.ptr) b.count = A.get(8, "a new-pair buffer");
    b.cap = cap;
    hip_check(sp::launch_fill_u64(b.count.as<unsigned long long>(), 1, 0, s), "fill");
}

// Grow a buffer to new_cap entries keeping [0, cap); its count becomes the
// old capacity (the entries there are pairs or holes).
void grow_buf(Buf &b, Alloc &A, uint64_t new_cap, hipStream_t s) {
    Mem k = A.get(new_cap * 4, "a new-pair buffer"), i = A.get(new_cap * 4, "a new-pair buffer"),
        j = A.get(new_cap * 4, "a new-pair buffer");
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

// What the seeding kernels read: the edges and the label -> matrix tables.
struct SeedInput {
    uint64_t m = 0;
    const uint32_t *src = nullptr, *dst = nullptr, *lab = nullptr;
    const uint32_t *lm_ptr = nullptr, *lm_mat = nullptr, *eps_mat = nullptr;
    uint32_t n_eps = 0;
    uint64_t max_seeds = 0;
};

// Slots of the seed buffer beyond the seeds: every wave of the two seeding
// kernels may leave one partly used chunk.
uint64_t seed_slack(uint64_t m, uint64_t eps_pairs) {
    auto waves = [](uint64_t items) {
        const uint64_t blocks = std::min<uint64_t>(std::max<uint64_t>(1, (items + 255) / 256), sp::kSeedBlocks);
        return items ? 4 * blocks : 0;
    };
    return (waves(m) + waves(eps_pairs)) * sp::kChunk;
}

// Thrown by sparse_core when the seeds of a mirror plan are not their own
// mirror image; solve_core then solves without the plan.
struct MirrorRejected {};

struct CoreOut {
    bool mirror = false;  // a mirror plan ran
    uint64_t mirror_skipped = 0;  // new pairs whose mirror the pass left out (counted in new_pairs)
    Mem dir, pool;  // the adjacency lists, kept for readout
    Mem hash, wit;  // the pair set and its witnesses, kept when witnesses are recorded
    uint64_t hash_slots = 0;
    Plan plan;
    uint32_t rounds = 0, reruns = 0;
    uint64_t seed_pairs = 0, new_pairs = 0, max_delta = 0, launches = 0;
    double product_ms = 0;
    // the heavy-bucket kernel of the grouped product (timing and accounting)
    double heavy_ms = 0, light_ms = 0, mirror_ms = 0;
    uint64_t heavy_launches = 0, heavy_bytes = 0, light_bytes = 0;
    bool timed_out = false;
};

// The solve.  A.fixed(): every structure is sized once from what the region
// leaves, and an overflow is an ENOMEM (nothing can grow); the key-sorted
// product (bucket arrays over all matrices and vertices) is off there.
void sparse_core(cflr_ctx *ctx, hipStream_t s, const cflr_opts &o, const Lowered &low, uint32_t n,
                 const SeedInput &in_seed, Alloc &A, CoreOut &res) {
    const bool fixed = A.fixed();
    const bool witness = o.witness != 0;
    if (witness && fixed) throw Error(CFLR_EUNSUPPORTED, "witnesses are not recorded by the no-alloc solve");
    if (witness && low.binary.size() >= sp::kWitEps)
        throw Error(CFLR_EUNSUPPORTED, "too many binary productions for witnesses");
    if (n >= sp::kMaxVertices) throw Error(CFLR_EUNSUPPORTED, "sparse storage holds at most 2^24 - 1 vertices");
    if (low.nmat() >= sp::kMaxMatrices) throw Error(CFLR_EUNSUPPORTED, "grammar needs 65535 or more matrices");
    const bool log = std::getenv("CFLR_LOG") != nullptr;
    auto too_small = [&](const char *what) {
        return Error(CFLR_ENOMEM, std::string("the no-alloc scratch cannot hold ") + what + " of this solve");
    };
    // a mirror plan when the grammar has a mirror (checked on the seeds below)
    std::vector<uint32_t> mirror_mat, mirror_rule;
    const bool mirrored = o.mirror != CFLR_MIRROR_OFF && find_mirror(low, &mirror_mat, &mirror_rule);
    if (!mirrored) mirror_rule.clear();
    if (!mirrored) mirror_mat.clear();
    res.plan = make_plan(low, n, mirror_rule, mirror_mat, !fixed);
    res.mirror = mirrored;
    const Plan &P = res.plan;
    Mem d_mirror, d_mirror_rule, d_mirror_ins;
    if (mirrored) {
        d_mirror = upload(A, mirror_mat, s, "the mirror tables");
        d_mirror_rule = upload(A, mirror_rule, s, "the mirror tables");
        // the pass leaves out mirrors that take no part in the rounds: no
        // uses, no lists of their own, head of no kept production (their
        // pairs are read out through their mirror's rows); with witnesses
        // every mirror is inserted (the readout looks each pair up)
        std::vector<uint32_t> ins(mirror_mat.size());
        for (uint32_t x = 0; x < (uint32_t)ins.size(); x++) {
            const uint32_t y = mirror_mat[x];
            const sp::MatInfo &my = P.mats[y];
            const bool inert = !witness && !my.nuse0 && !my.nuse1 && my.app_row == kNone && my.app_col == kNone &&
                               !P.kept_head[y];
            ins[x] = inert ? kNone : y;
        }
        d_mirror_ins = upload(A, ins, s, "the mirror tables");
    }

    Mem d_mats = upload(A, P.mats, s, "the matrix table");
    Mem d_uses = upload(A, P.uses, s, "the use table");
    Mem d_obs_ptr = upload(A, P.obs_ptr, s, "the observer table");
    Mem d_obs = upload(A, P.obs, s, "the observer table");
    const uint64_t cells = (uint64_t)P.nlayouts * n;
    res.dir = A.get(cells * sizeof(sp::Dir), "the list directory");
    Mem d_cur = A.get(cells * 4, "the list cursors");
    Mem d_mask = A.get(P.mask_words * 8, "the use masks");
    Mem d_ctl = A.get(sp::kCtlWords * 8, "the control words");
    if (cells) {
        hip_check(sp::launch_fill_u64(res.dir.as<unsigned long long>(), cells * 2, 0, s), "fill");
        hip_check(sp::launch_fill_u32(d_cur.as<uint32_t>(), cells, 0, s), "fill");
    }
    if (P.mask_words) hip_check(sp::launch_fill_u64(d_mask.as<unsigned long long>(), P.mask_words, 0, s), "fill");
    hip_check(sp::launch_fill_u64(d_ctl.as<unsigned long long>(), sp::kCtlWords, 0, s), "fill");

    const uint32_t grid = std::max<uint32_t>(1, ctx->num_cu * 8);
    uint32_t waves = o.grid_waves ? o.grid_waves : ctx->grid_waves_tuned;
    if (!waves) waves = ctx->num_cu * 32;
    if (fixed) waves = std::min<uint32_t>(waves, ctx->num_cu * 4);  // less chunk slack in a small region
    const uint64_t slack = 2ull * waves * 64;                       // keys a halted round may insert and take back
    const uint64_t out_slack = (uint64_t)waves * sp::kChunk;        // chunk slots a product may leave unused

    // capacities: the new-pair buffers (the first holds the seeds), the
    // list pool, the hash set; from earlier solves on this context (bounded
    // by the size of this input) or opts.delta_capacity -- or, in a fixed
    // region, split from what it leaves
    const uint64_t seeds_max = in_seed.max_seeds;
    const uint64_t seed_cap = seeds_max + seed_slack(in_seed.m, (uint64_t)in_seed.n_eps * n);
    const uint64_t scale = std::max<uint64_t>(1ull << 16, 4096 * seeds_max);
    uint64_t cap_out, pool_cap, slots = 0;
    uint64_t fixed_mark = 0;
    if (fixed) {
        // list pool 40 %, hash set 40 %, the two new-pair buffers with
        // their touched-list and copy queues the rest (52 bytes a pair)
        const uint64_t R = A.left() > (1u << 20) ? A.left() - (1u << 20) : 0;
        slots = pow2_at_most(std::max<uint64_t>(1, R * 2 / 5 / 8));
        pool_cap = R * 2 / 5 / 4;
        cap_out = R / 5 / 52;
        if (cap_out < seed_cap || cap_out <= out_slack) throw too_small("the seeds");
    } else {
        cap_out = o.delta_capacity ? std::max<uint64_t>(64, o.delta_capacity)
                                   : std::max<uint64_t>(1ull << 16, std::min(ctx->sparse_delta_hint, scale));
        pool_cap = std::max<uint64_t>(1ull << 20, 4 * seeds_max);
        if (!o.delta_capacity) pool_cap = std::max(pool_cap, std::min(ctx->sparse_pool_hint, 16 * scale));
    }
    Mem d_pool = A.get(pool_cap * 4, "the list pool");
    if (fixed) fixed_mark = A.mark();  // everything after this is free again after the solve
    Buf BA, BB;
    alloc_buf(BA, A, fixed ? cap_out : std::max(cap_out, seed_cap), s);
    alloc_buf(BB, A, cap_out, s);

    // hash set: at most 70 % full, counting what the next round may add
    uint64_t hash_keys = 0;       // pairs in the table
    uint64_t tombs_resident = 0;  // tombstones in the table (a rehash drops them)
    uint64_t cur_slots = 0;
    Mem hash, wit;
    auto hash_need = [&](uint64_t extra) {
        return pow2_at_least((hash_keys + tombs_resident + extra + slack) * 10 / 7 + 1);
    };
    sp::State S{};
    S.ctl = d_ctl.as<unsigned long long>();
    auto rehash_to = [&](uint64_t new_slots) {
        if (new_slots & (new_slots - 1)) throw Error(CFLR_EDEVICE, "internal: hash slots not a power of two");
        if (fixed && cur_slots) throw too_small("the pairs");
        Mem nh = A.get(new_slots * 8, "the hash set");
        hip_check(sp::launch_fill_u64(nh.as<unsigned long long>(), new_slots, sp::kEmpty, s), "fill");
        Mem nw;
        if (witness) nw = A.get(new_slots * 8, "the witnesses");
        if (cur_slots) {
            S.hash = nh.as<unsigned long long>();
            S.hash_mask = new_slots - 1;
            S.wit = witness ? nw.as<unsigned long long>() : nullptr;
            hip_check(sp::launch_rehash(S, hash.as<unsigned long long>(), witness ? wit.as<unsigned long long>() : nullptr,
                                        cur_slots, s),
                      "rehash");
        }
        hash = std::move(nh);
        if (witness) wit = std::move(nw);
        cur_slots = new_slots;
        S.hash = hash.as<unsigned long long>();
        S.hash_mask = cur_slots - 1;
        S.wit = witness ? wit.as<unsigned long long>() : nullptr;
        tombs_resident = 0;
        hip_check(sp::launch_fill_u64(S.ctl + sp::kCtlTomb, 1, 0, s), "fill");
    };

    Mem d_touched, d_moves;
    uint64_t touched_cap = 0;
    auto size_touched = [&](uint64_t in_cap) {
        if (touched_cap >= 2 * in_cap) return;
        touched_cap = 2 * in_cap;
        d_touched = A.get(touched_cap * 8, "the touched lists");
        d_moves = A.get(std::max<uint64_t>(1, touched_cap / 4) * 24, "the list copy queue");
    };
    if (fixed) size_touched(cap_out);

    // the grouped product: new pairs sorted by (matrix, key); buckets whose
    // products reach `threshold` are expanded into an LDS bit set, where a
    // use with at most `direct` products skips the bit set and a head's own
    // pairs are cleared from it when they are at most `row_factor` times
    // the use's products.  Defaults (128, 256, 4) from sweeps on the
    // 200,000-vertex points-to graph: the bit set and the own-row clear
    // replace most hash probes, and below these sizes a probe is cheaper
    // than the workgroup's fixed cost per use.  Off when the bucket space or
    // the bit set is too large, and in a fixed region.
    sp::KeySort K{};
    K.nb0 = (uint64_t)P.nrank0 * n;
    K.nb = K.nb0 + (uint64_t)P.nrank1 * n;
    const bool grouped = !fixed && K.nb > 0 && K.nb < (1ull << 30) && sp::heavy_lds_bytes(n) <= sp::kHeavyMaxLds &&
                         std::getenv("CFLR_SPARSE_UNGROUPED") == nullptr;
    uint64_t threshold = o.sparse_heavy ? o.sparse_heavy : (ctx->sparse_heavy_tuned ? ctx->sparse_heavy_tuned : 128);
    if (const char *h = std::getenv("CFLR_SPARSE_HEAVY")) threshold = std::max<uint64_t>(1, std::strtoull(h, nullptr, 10));
    if (witness) threshold = ~0ull;  // every product keeps its midpoint: no bucket goes to the bit set
    K.threshold = threshold;
    K.direct = 256;
    if (const char *h = std::getenv("CFLR_SPARSE_DIRECT")) K.direct = (uint32_t)std::strtoul(h, nullptr, 10);
    K.row_factor = 4;
    if (const char *h = std::getenv("CFLR_SPARSE_ROWF")) K.row_factor = (uint32_t)std::strtoul(h, nullptr, 10);
    Mem k_start, k_work, k_bsum, k_entry, k_heavy, k_light, k_ework, k_touch, k_acct;
    if (grouped) {
        k_start = A.get((K.nb + 1) * 4, "the key sort");
        k_work = A.get(K.nb * 8, "the key sort");
        k_bsum = A.get(sp::key_sort_scan_blocks(K.nb) * 4, "the key sort");
        K.start = k_start.as<uint32_t>();
        K.work = k_work.as<unsigned long long>();
        K.bsum = k_bsum.as<uint32_t>();
        if (o.count_traffic) {
            k_touch = A.get((cells + 31) / 32 * 4, "the traffic accounting");
            k_acct = A.get(16, "the traffic accounting");
            K.touch = k_touch.as<uint32_t>();
            K.acct = k_acct.as<unsigned long long>();
            K.acct_light = K.acct + 1;
        }
    }

    S.n = n;
    S.nlayouts = P.nlayouts;
    S.mats = d_mats.as<sp::MatInfo>();
    S.uses = d_uses.as<sp::Use>();
    S.obs_ptr = d_obs_ptr.as<uint32_t>();
    S.obs = d_obs.as<sp::Obs>();
    S.dir = res.dir.as<sp::Dir>();
    S.cur = d_cur.as<uint32_t>();
    S.mask = d_mask.as<uint64_t>();
    S.pool = d_pool.as<uint32_t>();
    S.pool_cap = pool_cap;
    if (fixed) {
        if (hash_need(seeds_max) > slots) throw too_small("the seeds");
        rehash_to(slots);
    } else {
        rehash_to(pow2_at_least(
            std::max(hash_need(seeds_max), o.delta_capacity ? 0 : std::min(ctx->sparse_slots_hint, 16 * scale))));
    }

    // control words read back after each step (pageable: no pinned allocation)
    unsigned long long h_ctl[sp::kCtlWords + 2] = {};
    auto read_ctl = [&](const Buf *out) {
        hip_check(hipMemcpyAsync(h_ctl, d_ctl.ptr, sp::kCtlWords * 8, hipMemcpyDeviceToHost, s), "D2H");
        if (out) hip_check(hipMemcpyAsync(h_ctl + sp::kCtlWords, out->count.ptr, 8, hipMemcpyDeviceToHost, s), "D2H");
        hip_check(hipStreamSynchronize(s), "sync");
    };
    auto clear_flags = [&](bool counters = true) {
        // halt, overflow flags and (counters) the product's counts; keep the
        // pool top and the tombstone count
        const int words[] = {sp::kCtlHalt,     sp::kCtlPoolOver,   sp::kCtlBufOver,         sp::kCtlHashFull,
                             sp::kCtlTasks,    sp::kCtlProducts,   sp::kCtlHeavyTasks,      sp::kCtlHeavyProducts,
                             sp::kCtlHeavyCand};
        for (int w : words) {
            if (!counters && w != sp::kCtlHalt && w != sp::kCtlPoolOver && w != sp::kCtlBufOver && w != sp::kCtlHashFull)
                continue;
            hip_check(sp::launch_fill_u64(S.ctl + w, 1, 0, s), "fill");
        }
    };

    // ---- seeds (a re-run after an overflow inserts only what is missing)
    hip_check(sp::launch_round_start(S, s), "round start");
    for (int attempt = 0;; attempt++) {
        hip_check(sp::launch_seed(S, in_seed.src, in_seed.dst, in_seed.lab, in_seed.m, in_seed.lm_ptr, in_seed.lm_mat,
                                  in_seed.eps_mat, in_seed.n_eps, BA.dev(), s),
                  "seed");
        read_ctl(&BA);
        if (!h_ctl[sp::kCtlHalt]) break;
        if (fixed) throw too_small("the seeds");
        if (attempt > 64) throw Error(CFLR_ENOMEM, "seeding keeps overflowing");
        if (h_ctl[sp::kCtlBufOver]) {
            const uint64_t asked = h_ctl[sp::kCtlWords];
            grow_buf(BA, A, std::max<uint64_t>(2 * BA.cap, asked + asked / 2), s);
        }
        const uint64_t resident = h_ctl[sp::kCtlNew] + h_ctl[sp::kCtlTomb];
        uint64_t want = pow2_at_least((resident + seeds_max + slack) * 10 / 7 + 1);
        if (h_ctl[sp::kCtlHashFull]) want = std::max(want, 2 * cur_slots);
        if (want > cur_slots) rehash_to(want);
        clear_flags();
    }
    if (mirrored) {
        // the seeds must be their own mirror image (the graph holds every
        // edge with its reverse); else the caller solves without the plan
        S.mirror = d_mirror.as<uint32_t>();
        S.mirror_rule = d_mirror_rule.as<uint32_t>();
        S.mirror_ins = d_mirror_ins.as<uint32_t>();
        hip_check(sp::launch_mirror_check(S, BA.dev(), std::min<uint64_t>(h_ctl[sp::kCtlWords], BA.cap), s),
                  "mirror check");
        read_ctl(nullptr);
        if (h_ctl[sp::kCtlMirrorMiss]) {
            if (log)
                std::fprintf(stderr, "[cflr] sparse: %llu seeds without their mirror; no mirror plan\n",
                             (unsigned long long)h_ctl[sp::kCtlMirrorMiss]);
            throw MirrorRejected{};
        }
    }
    uint64_t pending = h_ctl[sp::kCtlNew];
    res.seed_pairs = pending;
    hash_keys += pending;
    tombs_resident += h_ctl[sp::kCtlTomb];
    hip_check(sp::launch_fill_u64(S.ctl + sp::kCtlTomb, 1, 0, s), "fill");

    Buf *in = &BA, *out = &BB;
    hipEvent_t ev0 = nullptr, evh = nullptr, ev1 = nullptr;
    struct EvFree {
        hipEvent_t *e[3];
        ~EvFree() {
            for (auto p : e)
                if (*p) (void)hipEventDestroy(*p);
        }
    } ev_guard{{&ev0, &evh, &ev1}};
    if (o.kernel_timing && !fixed) {
        hip_check(hipEventCreate(&ev0), "event");
        hip_check(hipEventCreate(&evh), "event");
        hip_check(hipEventCreate(&ev1), "event");
    }
    while (pending) {
        if (o.max_rounds && res.rounds >= o.max_rounds) {
            res.timed_out = true;
            break;
        }
        res.rounds++;
        S.round = res.rounds;
        // room for this round: hash load, touched lists, the output buffer
        const uint64_t want_slots = hash_need(out->cap);
        if (want_slots > cur_slots) {
            if (fixed) throw too_small("the pairs");
            rehash_to(want_slots);
        }
        size_touched(in->cap);
        S.touched = d_touched.as<uint64_t>();
        S.touched_cap = touched_cap;
        S.moves = d_moves.as<uint64_t>();
        S.moves_cap = std::max<uint64_t>(1, touched_cap / 4);
        hip_check(sp::launch_fill_u64(out->count.as<unsigned long long>(), 1, 0, s), "fill");
        hip_check(sp::launch_round_start(S, s), "round start");

        // the key sort's arrays for this round's pairs (its bucket counts are
        // taken in the integration's pass)
        if (grouped && K.entry_cap < 2 * in->cap) {
            if (2 * in->cap >= (1ull << 32)) throw Error(CFLR_ENOMEM, "more than 2^31 new pairs in one round");
            K.entry_cap = K.heavy_cap = K.light_cap = 2 * in->cap;
            k_entry = A.get(K.entry_cap * 8, "the key sort");
            k_heavy = A.get(K.heavy_cap * 4, "the key sort");
            k_light = A.get(K.light_cap * 4, "the key sort");
            k_ework = A.get(K.entry_cap * 4, "the key sort");
            K.entry = k_entry.as<uint64_t>();
            K.heavy = k_heavy.as<uint32_t>();
            K.light = k_light.as<uint32_t>();
            K.ework = k_ework.as<uint32_t>();
        }
        const sp::KeySort *Kp = grouped ? &K : nullptr;

        // integrate the pending pairs into the lists
        hip_check(sp::launch_integrate(S, in->dev(), Kp, false, grid, s), "integrate");
        read_ctl(nullptr);
        while (h_ctl[sp::kCtlHalt]) {
            if (h_ctl[sp::kCtlTouchedOver]) throw Error(CFLR_EDEVICE, "internal: touched-list array too small");
            if (!h_ctl[sp::kCtlPoolOver]) throw Error(CFLR_EDEVICE, "internal: integration halted");
            if (fixed) throw too_small("the adjacency lists");
            const uint64_t top = h_ctl[sp::kCtlPoolTop], need = top + h_ctl[sp::kCtlAlloc];
            const uint64_t ncap = std::max<uint64_t>(2 * pool_cap, need + need / 2);
            Mem np = A.get(ncap * 4, "the list pool");
            hip_check(hipMemcpyAsync(np.ptr, d_pool.ptr, top * 4, hipMemcpyDeviceToDevice, s), "D2D");
            hip_check(hipStreamSynchronize(s), "sync");
            d_pool = std::move(np);
            pool_cap = ncap;
            S.pool = d_pool.as<uint32_t>();
            S.pool_cap = pool_cap;
            if (log) std::fprintf(stderr, "[cflr] sparse: pool grown to %llu entries\n", (unsigned long long)ncap);
            clear_flags();
            hip_check(sp::launch_integrate(S, in->dev(), Kp, true, grid, s), "integrate");
            read_ctl(nullptr);
        }
        hip_check(sp::launch_integrate_finish(S, in->dev(), Kp, grid, s), "integrate");

        // the product (a pool past kHeavyMaxPool entries sends every bucket to
        // the light kernel)
        if (grouped) {
            K.threshold = pool_cap <= sp::kHeavyMaxPool ? threshold : ~0ull;
            hip_check(sp::launch_key_sort(S, in->dev(), K, s), "key sort");
        }
        auto timed_product = [&]() {
            if (K.acct) {
                hip_check(sp::launch_fill_u32(K.touch, (cells + 31) / 32, 0, s), "fill");
                hip_check(sp::launch_fill_u64(K.acct, 2, 0, s), "fill");
            }
            if (ev0) hip_check(hipEventRecord(ev0, s), "event");
            if (grouped) {
                hip_check(sp::launch_heavy(S, K, out->dev(), waves, s), "product");
                if (evh) hip_check(hipEventRecord(evh, s), "event");
                hip_check(sp::launch_light(S, K, out->dev(), waves, s), "product");
                res.heavy_launches++;
            } else {
                hip_check(sp::launch_product(S, in->dev(), out->dev(), waves, s), "product");
            }
            if (ev1) hip_check(hipEventRecord(ev1, s), "event");
            res.launches++;
            read_ctl(out);
            if (ev1) {
                float ms = 0;
                hip_check(hipEventElapsedTime(&ms, ev0, ev1), "event");
                res.product_ms += ms;
                if (grouped) {
                    float hm = 0;
                    hip_check(hipEventElapsedTime(&hm, ev0, evh), "event");
                    res.heavy_ms += hm;
                    res.light_ms += ms - hm;
                }
            }
            if (K.acct) {
                unsigned long long b[2] = {0, 0};
                copy_sync(b, K.acct, 16, hipMemcpyDeviceToHost, s);
                res.heavy_bytes += b[0];
                res.light_bytes += b[1];
            }
        };
        hip_check(sp::launch_fill_u64(S.ctl + sp::kCtlNew, 1, 0, s), "fill");
        hip_check(sp::launch_fill_u64(S.ctl + sp::kCtlProducts, 1, 0, s), "fill");
        hip_check(sp::launch_fill_u64(S.ctl + sp::kCtlHeavyProducts, 2, 0, s), "fill");
        const double heavy_ms0 = res.heavy_ms, light_ms0 = res.light_ms, mirror_ms0 = res.mirror_ms;
        const uint64_t heavy_b0 = res.heavy_bytes, light_b0 = res.light_bytes;
        // an overflow halted the step: grow what overflowed before re-running it
        auto grow_for_rerun = [&](int attempt, const char *step, bool counters) {
            if (fixed) throw too_small("the pairs");
            if (attempt > 64) throw Error(CFLR_ENOMEM, "new-pair buffer or hash set keeps overflowing");
            res.reruns++;
            if (h_ctl[sp::kCtlBufOver]) {
                const uint64_t asked = h_ctl[sp::kCtlWords];
                const uint64_t ncap = std::max<uint64_t>(2 * out->cap, asked + asked / 2);
                if (ncap > (1ull << 34)) throw Error(CFLR_ENOMEM, "new-pair buffer beyond 2^34 pairs");
                grow_buf(*out, A, ncap, s);
            }
            // the table holds the pairs appended so far this round and the
            // tombstones of the halted run: room for what the re-run may add
            const uint64_t resident = hash_keys + h_ctl[sp::kCtlNew] + tombs_resident + h_ctl[sp::kCtlTomb];
            uint64_t want = pow2_at_least((resident + out->cap + slack) * 10 / 7 + 1);
            if (h_ctl[sp::kCtlHashFull]) want = std::max(want, 2 * cur_slots);
            if (want > cur_slots) rehash_to(want);  // drops the tombstones
            if (log)
                std::fprintf(stderr, "[cflr] sparse: round %u %s re-run (buffer %llu, slots %llu)\n", res.rounds, step,
                             (unsigned long long)out->cap, (unsigned long long)cur_slots);
            clear_flags(counters);
        };
        timed_product();
        for (int attempt = 0; h_ctl[sp::kCtlHalt]; attempt++) {
            grow_for_rerun(attempt, "product", true);
            timed_product();
        }
        if (mirrored) {
            // the mirrors of the product's pairs, appended behind them
            const uint64_t nprod = std::min<uint64_t>(h_ctl[sp::kCtlWords], out->cap);
            if (ev0) hip_check(hipEventRecord(ev0, s), "event");
            hip_check(sp::launch_fill_u64(S.ctl + sp::kCtlMirrorSkip, 1, 0, s), "fill");
            hip_check(sp::launch_mirror(S, out->dev(), nprod, waves, s), "mirror");
            read_ctl(out);
            for (int attempt = 0; h_ctl[sp::kCtlHalt]; attempt++) {
                grow_for_rerun(attempt, "mirror pass", false);
                hip_check(sp::launch_fill_u64(S.ctl + sp::kCtlMirrorSkip, 1, 0, s), "fill");
                hip_check(sp::launch_mirror(S, out->dev(), nprod, waves, s), "mirror");
                read_ctl(out);
            }
            res.mirror_skipped += h_ctl[sp::kCtlMirrorSkip];
            if (ev0) {
                hip_check(hipEventRecord(ev1, s), "event");
                hip_check(hipEventSynchronize(ev1), "event");
                float ms = 0;
                hip_check(hipEventElapsedTime(&ms, ev0, ev1), "event");
                res.mirror_ms += ms;
                res.product_ms += ms;
            }
        }
        // kCtlNew counts every pair appended this round, over re-runs too
        const uint64_t fresh = h_ctl[sp::kCtlNew];
        res.new_pairs += fresh + (mirrored ? h_ctl[sp::kCtlMirrorSkip] : 0);
        hash_keys += fresh;
        tombs_resident += h_ctl[sp::kCtlTomb];
        hip_check(sp::launch_fill_u64(S.ctl + sp::kCtlTomb, 1, 0, s), "fill");
        res.max_delta = std::max(res.max_delta, fresh);
        if (log)
            std::fprintf(stderr,
                         "[cflr] sparse round %u: in %llu new %llu products %llu heavy items %llu products %llu "
                         "candidates %llu pool %llu/%llu slots %llu heavy %.2f ms light %.2f ms mirror %.2f ms "
                         "algo bytes heavy %llu light %llu\n",
                         res.rounds, (unsigned long long)pending, (unsigned long long)fresh,
                         (unsigned long long)h_ctl[sp::kCtlProducts], (unsigned long long)h_ctl[sp::kCtlHeavy],
                         (unsigned long long)h_ctl[sp::kCtlHeavyProducts], (unsigned long long)h_ctl[sp::kCtlHeavyCand],
                         (unsigned long long)h_ctl[sp::kCtlPoolTop], (unsigned long long)pool_cap,
                         (unsigned long long)cur_slots, res.heavy_ms - heavy_ms0, res.light_ms - light_ms0,
                         res.mirror_ms - mirror_ms0,
                         (unsigned long long)(res.heavy_bytes - heavy_b0),
                         (unsigned long long)(res.light_bytes - light_b0));
        pending = fresh;
        std::swap(in, out);
    }
    if (!pending && !res.timed_out) res.rounds++;  // the round that derived nothing (counted as the dense engine does)
    if (!fixed) {
        ctx->sparse_delta_hint = std::max({ctx->sparse_delta_hint, BA.cap, BB.cap});
        ctx->sparse_pool_hint = std::max(ctx->sparse_pool_hint, pool_cap);
        ctx->sparse_slots_hint = std::max(ctx->sparse_slots_hint, cur_slots);
    }
    res.pool = std::move(d_pool);
    if (witness) {
        res.hash = std::move(hash);
        res.wit = std::move(wit);
        res.hash_slots = cur_slots;
    }
    if (fixed) {
        hip_check(hipStreamSynchronize(s), "sync");
        A.release_to(fixed_mark);  // the hash set, buffers and queues are free again (readout scratch)
    }
}

// sparse_core with a mirror plan when one applies; when the seeds reject
// it, again without (from the same point of the region, in a fixed one).
void solve_core(cflr_ctx *ctx, hipStream_t s, const cflr_opts &o, const Lowered &low, uint32_t n,
                const SeedInput &in_seed, Alloc &A, CoreOut &res) {
    if (o.mirror != CFLR_MIRROR_OFF) {
        const uint64_t mark = A.fixed() ? A.mark() : 0;
        try {
            sparse_core(ctx, s, o, low, n, in_seed, A, res);
            return;
        } catch (const MirrorRejected &) {
            res = CoreOut{};
            if (A.fixed()) A.release_to(mark);
        }
    }
    cflr_opts off = o;
    off.mirror = CFLR_MIRROR_OFF;
    sparse_core(ctx, s, off, low, n, in_seed, A, res);
}

// Graph label -> the matrices x with x -> label (after lowering), as
// offsets and a flat list; also the most matrices one label seeds.
void label_tables(const Lowered &low, const std::vector<std::string> &label_names, std::vector<uint32_t> *ptr,
                  std::vector<uint32_t> *mats, uint32_t *max_per_label) {
    std::map<std::string, uint32_t> term_id;
    for (uint32_t t = 0; t < low.terminals.size(); t++) term_id[low.terminals[t]] = t;
    std::vector<std::vector<uint32_t>> by_term(low.terminals.size());
    for (auto &tm : low.term) by_term[tm.first].push_back(tm.second);
    const uint32_t L = (uint32_t)label_names.size();
    ptr->assign(L + 1, 0);
    mats->clear();
    *max_per_label = 0;
    for (uint32_t l = 0; l < L; l++) {
        auto it = term_id.find(label_names[l]);
        if (it != term_id.end())
            for (uint32_t x : by_term[it->second]) mats->push_back(x);
        (*ptr)[l + 1] = (uint32_t)mats->size();
        *max_per_label = std::max(*max_per_label, (*ptr)[l + 1] - (*ptr)[l]);
    }
}

}  // namespace

// ------------------------------------------------------------------- solve

uint32_t mirror_skipped(const Lowered &low) {
    std::vector<uint32_t> mat, rule;
    if (!find_mirror(low, &mat, &rule)) return 0;
    uint32_t k = 0;
    for (uint32_t q = 0; q < (uint32_t)rule.size(); q++) k += rule[q] < q;
    return k;
}


void sparse_solve(cflr_ctx *ctx, const cflr_opts &o, Instance &inst, bool *timed_out, hipStream_t stream) {
    Alloc A(ctx->pool.get());
    SeedInput in;
    in.m = inst.graph->m;
    in.src = inst.graph->src.as<uint32_t>();
    in.dst = inst.graph->dst.as<uint32_t>();
    in.lab = inst.graph->lab.as<uint32_t>();
    in.lm_ptr = inst.lm_ptr.as<uint32_t>();
    in.lm_mat = inst.lm_mat.as<uint32_t>();
    in.eps_mat = inst.eps_mat.as<uint32_t>();
    in.n_eps = inst.n_eps;
    in.max_seeds = inst.max_seeds;
    CoreOut res;
    solve_core(ctx, stream ? stream : ctx->stream, o, inst.low, inst.n, in, A, res);
    *timed_out = res.timed_out;
    auto store = std::make_shared<SparseStore>();
    store->hold = CtxRef(ctx);
    store->ctx = ctx;
    store->n = inst.n;
    store->nlayouts = res.plan.nlayouts;
    store->row_layout.resize(inst.low.nmat());
    for (uint32_t x = 0; x < inst.low.nmat(); x++) store->row_layout[x] = res.plan.mats[x].row_layout;
    store->readout_mirror = res.plan.readout_mirror;
    store->dir = std::move(res.dir.buf);
    store->pool = std::move(res.pool.buf);
    if (o.witness) {
        store->hash = std::move(res.hash.buf);
        store->wit = std::move(res.wit.buf);
        store->hash_slots = res.hash_slots;
        // symbols: user non-terminals, then U + terminal index
        const Lowered &low = inst.low;
        const uint32_t U = (uint32_t)low.user_names.size();
        std::vector<uint32_t> sym(low.nmat(), CFLR_NONE);
        for (uint32_t x = 0; x < U; x++) sym[x] = x;
        for (auto &tm : low.term)
            if (tm.second >= U) sym[tm.second] = U + tm.first;  // a wrapper T_t -> t stands for t
        for (auto &b : low.binary) {
            store->prod_sym.push_back(sym[b.a]);
            store->prod_sym.push_back(sym[b.b]);
        }
        std::map<std::string, uint32_t> term_id;
        for (uint32_t t = 0; t < low.terminals.size(); t++) term_id[low.terminals[t]] = t;
        for (auto &name : inst.graph->label_names) {
            auto it = term_id.find(name);
            store->label_sym.push_back(it == term_id.end() ? CFLR_NONE : U + it->second);
        }
    }
    inst.rounds = res.rounds;
    inst.done = !res.timed_out;
    inst.stats.rounds = res.rounds;
    inst.stats.reruns = res.reruns;
    inst.stats.seed_pairs = res.seed_pairs;
    inst.stats.new_pairs = res.new_pairs;
    inst.stats.max_delta = res.max_delta;
    inst.stats.product_ms = res.product_ms;
    inst.stats.product_launches = res.launches;
    inst.stats.heavy_ms = res.heavy_ms;
    inst.stats.heavy_launches = res.heavy_launches;
    inst.stats.heavy_algo_bytes = res.heavy_bytes;
    inst.stats.light_ms = res.light_ms;
    inst.stats.light_algo_bytes = res.light_bytes;
    inst.stats.mirror = res.mirror ? 1 : 0;
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
    for (uint32_t x = 0; x < U; x++) {
        const uint32_t from = st.readout_mirror[x] == kNone ? x : st.readout_mirror[x];  // equal counts
        hip_check(sp::launch_layout_count(st.dir.as<sp::Dir>() + (uint64_t)st.row_layout[from] * st.n, st.n,
                                          tot.as<unsigned long long>() + x, s),
                  "count");
    }
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
    const sp::Dir *dir = nullptr;
    const uint32_t *lists = st.pool.as<uint32_t>();
    DevBuf tdir, tpool;
    if (st.readout_mirror[nt] == kNone) {
        dir = st.dir.as<sp::Dir>() + (uint64_t)st.row_layout[nt] * n;
    } else {
        // nt's pairs are its mirror's rows transposed: count the entries per
        // column, lay the columns out as lists, fill them, then read those
        // lists as rows
        const sp::Dir *mdir = st.dir.as<sp::Dir>() + (uint64_t)st.row_layout[st.readout_mirror[nt]] * n;
        DevBuf cnt(pool, (uint64_t)n * 4), cur(pool, (uint64_t)n * 4);
        hip_check(hipMemsetAsync(cnt.ptr, 0, (uint64_t)n * 4, s), "memset");
        hip_check(hipMemsetAsync(cur.ptr, 0, (uint64_t)n * 4, s), "memset");
        hip_check(sp::launch_transpose_count(mdir, st.pool.as<uint32_t>(), n, cnt.as<uint32_t>(), s), "readout");
        std::vector<uint32_t> hc(n);
        copy_sync(hc.data(), cnt.ptr, (uint64_t)n * 4, hipMemcpyDeviceToHost, s);
        std::vector<sp::Dir> td(n);
        uint64_t at = 0;
        for (uint32_t j = 0; j < n; j++) {
            td[j] = sp::Dir{at, hc[j], hc[j]};
            at += hc[j];
        }
        if (at != count) throw Error(CFLR_EDEVICE, "internal: transposed readout count differs");
        tdir = DevBuf(pool, (uint64_t)n * sizeof(sp::Dir));
        tpool = DevBuf(pool, std::max<uint64_t>(1, at) * 4);
        copy_sync(tdir.ptr, td.data(), (uint64_t)n * sizeof(sp::Dir), hipMemcpyHostToDevice, s);
        hip_check(sp::launch_transpose_scatter(mdir, st.pool.as<uint32_t>(), n, tdir.as<sp::Dir>(),
                                               cur.as<uint32_t>(), tpool.as<uint32_t>(), s),
                  "readout");
        dir = tdir.as<sp::Dir>();
        lists = tpool.as<uint32_t>();
    }
    if (on_device) {
        hip_check(sp::launch_layout_write(dir, lists, n, off.as<uint64_t>(), bm.as<uint64_t>(), sort_grid, src, dst, s),
                  "readout");
        hip_check(hipStreamSynchronize(s), "sync");
        return;
    }
    DevBuf dsrc(pool, count * 4), ddst(pool, count * 4);
    hip_check(sp::launch_layout_write(dir, lists, n, off.as<uint64_t>(), bm.as<uint64_t>(), sort_grid,
                                      dsrc.as<uint32_t>(), ddst.as<uint32_t>(), s),
              "readout");
    hip_check(hipMemcpyAsync(src, dsrc.ptr, count * 4, hipMemcpyDeviceToHost, s), "D2H");
    hip_check(hipMemcpyAsync(dst, ddst.ptr, count * 4, hipMemcpyDeviceToHost, s), "D2H");
    hip_check(hipStreamSynchronize(s), "sync");
}

void sparse_witness(Instance &inst, uint32_t nt, uint32_t *left, uint32_t *right, uint32_t *mid, uint32_t *round,
                    uint64_t count, bool on_device) {
    SparseStore &st = *inst.sp;
    if (!st.hash_slots) throw Error(CFLR_EINVAL, "no witnesses: solve with cflr_opts.witness = 1");
    if (!count) return;
    cflr_ctx *ctx = inst.ctx;
    hipStream_t s = ctx->stream;
    DevPool *pool = ctx->pool.get();
    DevBuf dsrc(pool, count * 4), ddst(pool, count * 4);
    sparse_copy(inst, nt, dsrc.as<uint32_t>(), ddst.as<uint32_t>(), count, true);
    const uint64_t np = std::max<size_t>(1, st.prod_sym.size()), nl = std::max<size_t>(1, st.label_sym.size());
    DevBuf psym(pool, np * 4), lsym(pool, nl * 4), miss(pool, 8);
    if (!st.prod_sym.empty())
        copy_sync(psym.ptr, st.prod_sym.data(), st.prod_sym.size() * 4, hipMemcpyHostToDevice, s);
    if (!st.label_sym.empty())
        copy_sync(lsym.ptr, st.label_sym.data(), st.label_sym.size() * 4, hipMemcpyHostToDevice, s);
    hip_check(sp::launch_fill_u64(miss.as<unsigned long long>(), 1, 0, s), "fill");
    DevBuf tl, tr, tm, td;
    uint32_t *L = left, *R = right, *Md = mid, *Rd = round;
    if (!on_device) {
        tl = DevBuf(pool, count * 4);
        tr = DevBuf(pool, count * 4);
        tm = DevBuf(pool, count * 4);
        td = DevBuf(pool, count * 4);
        L = tl.as<uint32_t>();
        R = tr.as<uint32_t>();
        Md = tm.as<uint32_t>();
        Rd = td.as<uint32_t>();
    }
    const uint32_t x = nt;  // user non-terminals are the first matrices
    hip_check(sp::launch_witness(st.hash.as<unsigned long long>(), st.hash_slots - 1, st.wit.as<unsigned long long>(),
                                 x, dsrc.as<uint32_t>(), ddst.as<uint32_t>(), count, psym.as<uint32_t>(),
                                 (uint32_t)(st.prod_sym.size() / 2), lsym.as<uint32_t>(),
                                 (uint32_t)st.label_sym.size(), L, R, Md, Rd, miss.as<unsigned long long>(), s),
              "witness");
    unsigned long long missing = 0;
    copy_sync(&missing, miss.ptr, 8, hipMemcpyDeviceToHost, s);
    if (missing) throw Error(CFLR_EDEVICE, "internal: a result pair has no witness in the pair set");
    if (!on_device) {
        hip_check(hipMemcpyAsync(left, L, count * 4, hipMemcpyDeviceToHost, s), "D2H");
        hip_check(hipMemcpyAsync(right, R, count * 4, hipMemcpyDeviceToHost, s), "D2H");
        hip_check(hipMemcpyAsync(mid, Md, count * 4, hipMemcpyDeviceToHost, s), "D2H");
        hip_check(hipMemcpyAsync(round, Rd, count * 4, hipMemcpyDeviceToHost, s), "D2H");
    }
    hip_check(hipStreamSynchronize(s), "sync");
}

// ------------------------------------------------------- no-alloc entry point

// The fixed device region of cflr_solve_noalloc.  In host code `scratch` is
// a stand-in for the symbol, not a device address: every use goes through
// the address hipGetSymbolAddress gives for the current device.
constexpr uint64_t kScratchBytes = CFLR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device -> its copy of `scratch`

// With the device current: the address of its `scratch`, looked up once.
void *scratch_address(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) return it->second;
    void *p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) throw Error(CFLR_EDEVICE, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_ptr[device] = p;
    return p;
}

}  // namespace

void sparse_solve_noalloc(cflr_ctx *ctx, const Lowered &low, uint32_t n, uint64_t m, const uint32_t *src,
                          const uint32_t *dst, const uint32_t *label, const std::vector<std::string> &label_names,
                          const cflr_opts &o, uint32_t *out_src, uint32_t *out_dst, uint64_t capacity,
                          uint64_t *counts, cflr_stats *stats) {
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = ctx->stream;
    Alloc A(scratch_address(ctx->device), kScratchBytes);
    // the seeding tables, and a check of the edges on the device
    std::vector<uint32_t> ptr, mats;
    uint32_t max_per_label = 0;
    label_tables(low, label_names, &ptr, &mats, &max_per_label);
    Mem lm_ptr = upload(A, ptr, s, "the label table");
    Mem lm_mat = upload(A, mats, s, "the label table");
    Mem eps_mat = upload(A, low.eps, s, "the eps table");
    if (m) {
        Mem bad = A.get(8, "the edge check");
        hip_check(sp::launch_fill_u64(bad.as<unsigned long long>(), 1, 0, s), "fill");
        hip_check(sp::launch_check_edges(src, dst, label, m, n, (uint32_t)label_names.size(),
                                         bad.as<unsigned long long>(), s),
                  "edge check");
        unsigned long long h = 0;
        copy_sync(&h, bad.ptr, 8, hipMemcpyDeviceToHost, s);
        if (h) throw Error(CFLR_EINVAL, "an edge has a vertex >= n or a label >= n_labels");
    }
    SeedInput in;
    in.m = m;
    in.src = src;
    in.dst = dst;
    in.lab = label;
    in.lm_ptr = lm_ptr.as<uint32_t>();
    in.lm_mat = lm_mat.as<uint32_t>();
    in.eps_mat = eps_mat.as<uint32_t>();
    in.n_eps = (uint32_t)low.eps.size();
    in.max_seeds = m * max_per_label + (uint64_t)n * in.n_eps;
    CoreOut res;
    solve_core(ctx, s, o, low, n, in, A, res);
    // readout into the caller's arrays, each non-terminal's pairs sorted by
    // (i, j), one after another in first-appearance order; the scratch
    // after the lists holds the counts, offsets and sort bit sets
    const uint32_t U = (uint32_t)low.user_names.size();
    Mem tot = A.get(8ull * std::max<uint32_t>(1, U), "the readout");
    hip_check(sp::launch_fill_u64(tot.as<unsigned long long>(), std::max<uint32_t>(1, U), 0, s), "fill");
    const sp::Dir *dir = res.dir.as<sp::Dir>();
    for (uint32_t x = 0; x < U; x++)
        hip_check(sp::launch_layout_count(dir + (uint64_t)res.plan.mats[x].row_layout * n, n,
                                          tot.as<unsigned long long>() + x, s),
                  "count");
    std::vector<unsigned long long> h(std::max<uint32_t>(1, U));
    copy_sync(h.data(), tot.ptr, 8ull * std::max<uint32_t>(1, U), hipMemcpyDeviceToHost, s);
    uint64_t total = 0;
    for (uint32_t x = 0; x < U; x++) {
        counts[x] = h[x];
        total += h[x];
    }
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->rounds = res.rounds;
        stats->seed_pairs = res.seed_pairs;
        stats->new_pairs = res.new_pairs;
        stats->total_pairs = total;
        stats->max_delta = res.max_delta;
        stats->product_launches = res.launches;
        stats->device_bytes = kScratchBytes;
        stats->storage = CFLR_STORAGE_SPARSE;
    }
    if (res.timed_out) throw Error(CFLR_ETIMEOUT, "round limit reached before the fixpoint (nothing written)");
    if (total > capacity)
        throw Error(CFLR_EINVAL, "capacity " + std::to_string(capacity) + " is smaller than the " +
                                     std::to_string(total) + " pairs (counts written, pairs not)");
    if (total && (!out_src || !out_dst)) throw Error(CFLR_EINVAL, "null output array");
    const uint32_t sort_grid = std::max<uint32_t>(1, std::min<uint32_t>(ctx->num_cu, std::max<uint32_t>(1, n)));
    const uint64_t nw = ((uint64_t)n + 63) / 64;
    Mem off = A.get((uint64_t)std::max<uint32_t>(1, n) * 8, "the readout");
    Mem bm = A.get((uint64_t)sort_grid * std::max<uint64_t>(1, nw) * 8, "the readout");
    hip_check(sp::launch_fill_u64(bm.as<unsigned long long>(), (uint64_t)sort_grid * std::max<uint64_t>(1, nw), 0, s),
              "fill");
    uint64_t at = 0;
    for (uint32_t x = 0; x < U; x++) {
        if (h[x])
            hip_check(sp::launch_layout_write(dir + (uint64_t)res.plan.mats[x].row_layout * n, res.pool.as<uint32_t>(),
                                              n, off.as<uint64_t>(), bm.as<uint64_t>(), sort_grid, out_src + at,
                                              out_dst + at, s),
                      "readout");
        at += h[x];
    }
    hip_check(hipStreamSynchronize(s), "sync");
    if (stats)
        stats->fixpoint_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace cflr

// sparse_kernels.hip -- kernels of the sparse storage engine (gfx950, wave64).
//
// A round of the semi-naive fixpoint (Section 3, optimisation 1) on pair
// storage (layout in sparse.h):
//
//   integrate  the previous round's new pairs are appended to the
//              adjacency lists of their matrix (count per list -> plan the
//              moves of lists that outgrow their block -> check the pool ->
//              move -> scatter), and lists that become non-empty set their
//              bit in the use masks of the productions that read them;
//   product    every new pair of a matrix x meets, for every production
//              using x whose mask bit is set at the pair's partner vertex,
//              the partner list: part 0 (x = a of c -> a b, new pair (i, k))
//              reads row k of b and yields (c, i, j); part 1 (x = b, new pair
//              (k, j)) reads column k of a and yields (c, i, j).  Each
//              candidate is inserted into the hash set; the inserts that
//              succeed are the round's new pairs of c (New_c = Cand \ M_c and
//              M_c <- M_c U New_c in one compare-and-swap).
//
// A wave expands the lists of its 64 lanes together: the lanes' list
// lengths are prefix-summed and each pass takes 64 consecutive products, a
// lane finding the list its product belongs to by a binary search over the
// prefix sums.  New pairs are appended in chunks reserved per wave.
#include <hip/hip_runtime.h>

#include "sparse.h"

namespace cflr {
namespace sp {

namespace {

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint32_t first_lane(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t first_lane64(uint64_t v) {
    return ((uint64_t)first_lane((uint32_t)(v >> 32)) << 32) | first_lane((uint32_t)v);
}

__device__ __forceinline__ uint32_t shfl32(uint32_t v, uint32_t l) { return (uint32_t)__shfl((int)v, (int)l, 64); }

__device__ __forceinline__ uint64_t shfl64(uint64_t v, uint32_t l) {
    return ((uint64_t)shfl32((uint32_t)(v >> 32), l) << 32) | shfl32((uint32_t)v, l);
}

// exclusive prefix sum over the wave; *total = sum over all lanes
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t *total) {
    const uint32_t lane = lane_id();
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, d, 64);
        if (lane >= (uint32_t)d) x += y;
    }
    *total = __builtin_amdgcn_readlane(x, 63);
    return x - v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
    for (int d = 32; d; d >>= 1) v += shfl64(v, lane_id() ^ (uint32_t)d);
    return v;
}

__device__ __forceinline__ unsigned long long load_relaxed(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 64-bit finaliser of SplitMix64 (Steele, Lea and Flood, 2014): spreads the
// packed (matrix, i, j) keys over the table.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

constexpr uint32_t kMaxProbes = 4096;  // the host keeps the load below 0.7
enum { kPresent = 0, kInserted = 1, kFull = 2 };

// Linear-probing insert.  kInserted: this thread added the key (its slot in
// *where); kPresent: the key was there (or another thread added it first);
// kFull: no free slot within kMaxProbes (the host re-runs after a rehash).
__device__ __forceinline__ int hash_insert(unsigned long long *tab, uint64_t hmask, uint64_t key, uint64_t *where) {
    uint64_t h = mix64(key) & hmask;
    for (uint32_t p = 0; p < kMaxProbes; p++) {
        const unsigned long long v = load_relaxed(&tab[h]);
        if (v == key) return kPresent;
        if (v == kEmpty) {
            const unsigned long long prev = atomicCAS(&tab[h], (unsigned long long)kEmpty, (unsigned long long)key);
            if (prev == kEmpty) {
                *where = h;
                return kInserted;
            }
            if (prev == key) return kPresent;
        }
        h = (h + 1) & hmask;
    }
    return kFull;
}

// Append slots of a new-pair buffer, reserved per wave in chunks so that one
// device-scope atomic serves many appends; unused slots of a chunk become
// holes when the wave moves on or exits (kChunk slots at a time).

struct Chunk {
    uint64_t pos = 0, end = 0;  // wave-uniform
};

__device__ __forceinline__ void chunk_retire(const PairBuf &B, Chunk &ch) {
    for (uint64_t x = ch.pos + lane_id(); x < ch.end; x += 64) B.key[x] = kHoleKey;
    ch.pos = ch.end;
}

// Every lane of the wave calls this together.  Lane l gets `need` slots at
// *pos.  false: the buffer is full (flags set, nothing reserved).
__device__ __forceinline__ bool chunk_reserve(const PairBuf &B, Chunk &ch, uint32_t need, uint64_t *pos,
                                              unsigned long long *ctl) {
    uint32_t total;
    const uint32_t pre = wave_excl_scan(need, &total);
    *pos = 0;
    if (!total) return true;
    if (ch.pos + total > ch.end) {
        chunk_retire(B, ch);
        const uint64_t want = total > kChunk ? total : kChunk;
        unsigned long long base = 0;
        if (lane_id() == 0) base = atomicAdd(B.count, (unsigned long long)want);
        base = first_lane64(base);
        if (base + want > B.cap) {
            for (uint64_t x = base + lane_id(); x < B.cap && x < base + want; x += 64) B.key[x] = kHoleKey;
            ch.pos = ch.end = 0;
            if (lane_id() == 0) {
                atomicOr(&ctl[kCtlBufOver], 1ull);
                atomicOr(&ctl[kCtlHalt], 1ull);
            }
            return false;
        }
        ch.pos = base;
        ch.end = base + want;
    }
    *pos = ch.pos + pre;
    ch.pos += total;
    return true;
}

// Insert (m, i, j) for the lanes with `has`; append the new ones and, when
// the solve keeps witnesses, record w for them.  Every lane calls this
// together.  false: an overflow (this wave's new keys of the call were
// taken back; the round is re-run).
__device__ __forceinline__ bool insert_append(const State &S, const PairBuf &out, Chunk &ch, uint64_t &appended,
                                              bool has, uint32_t m, uint32_t i, uint32_t j, uint64_t w) {
    int ins = kPresent;
    uint64_t where = 0;
    if (has) ins = hash_insert(S.hash, S.hash_mask, pair_key(m, i, j), &where);
    const bool full = __any(ins == kFull);
    uint64_t pos = 0;
    bool ok = !full;
    if (ok) ok = chunk_reserve(out, ch, ins == kInserted ? 1u : 0u, &pos, S.ctl);
    if (!ok) {
        if (ins == kInserted) {
            atomicExch(&S.hash[where], (unsigned long long)kTomb);
            atomicAdd(&S.ctl[kCtlTomb], 1ull);
        }
        if (full && lane_id() == 0) {
            atomicOr(&S.ctl[kCtlHashFull], 1ull);
            atomicOr(&S.ctl[kCtlHalt], 1ull);
        }
        return false;
    }
    if (ins == kInserted) {
        out.key[pos] = m;
        out.i[pos] = i;
        out.j[pos] = j;
        if (S.wit) S.wit[where] = w;
    }
    appended += (uint64_t)__popcll(__ballot(ins == kInserted));
    return true;
}

// A wave's count of appended pairs, added once when it exits.
__device__ __forceinline__ void add_appended(const State &S, uint64_t appended) {
    if (lane_id() == 0 && appended) atomicAdd(&S.ctl[kCtlNew], (unsigned long long)appended);
}

// Lanes with `want` take consecutive slots of a device counter: one atomic
// per wave; every lane calls this together.  Returns the lane's slot (valid
// where want).
__device__ __forceinline__ uint64_t wave_reserve(unsigned long long *ctr, bool want) {
    const uint64_t mask = __ballot(want);
    if (!mask) return 0;
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(ctr, (unsigned long long)__popcll(mask));
    base = first_lane64(base);
    return base + (uint64_t)__popcll(mask & ((1ull << lane_id()) - 1));
}

__device__ __forceinline__ uint64_t wave_global_id() {
    return ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
}
__device__ __forceinline__ uint64_t waves_in_grid() { return ((uint64_t)gridDim.x * blockDim.x) / 64; }

}  // namespace

// ------------------------------------------------------------------ seeding

__global__ __launch_bounds__(256) void seed_edges_kernel(State S, const uint32_t *src, const uint32_t *dst,
                                                         const uint32_t *lab, uint64_t m, const uint32_t *lm_ptr,
                                                         const uint32_t *lm_mat, PairBuf out) {
    Chunk ch;
    uint64_t appended = 0;
    for (uint64_t base = wave_global_id() * 64; base < m; base += waves_in_grid() * 64) {
        const uint64_t e = base + lane_id();
        uint32_t q0 = 0, q1 = 0, u = 0, v = 0;
        if (e < m) {
            const uint32_t l = lab[e];
            q0 = lm_ptr[l];
            q1 = lm_ptr[l + 1];
            u = src[e];
            v = dst[e];
        }
        for (uint32_t q = q0;; q++) {
            const bool has = q < q1;
            if (!__any(has)) break;
            if (!insert_append(S, out, ch, appended, has, has ? lm_mat[q] : 0u, u, v,
                               make_witness(0, kWitEdge, e < m ? lab[e] : 0u))) {
                add_appended(S, appended);
                return;
            }
        }
    }
    chunk_retire(out, ch);
    add_appended(S, appended);
}

__global__ __launch_bounds__(256) void seed_eps_kernel(State S, const uint32_t *eps_mat, uint32_t n_eps,
                                                       PairBuf out) {
    Chunk ch;
    uint64_t appended = 0;
    const uint64_t total = (uint64_t)n_eps * S.n;
    for (uint64_t base = wave_global_id() * 64; base < total; base += waves_in_grid() * 64) {
        const uint64_t x = base + lane_id();
        const bool has = x < total;
        const uint32_t e = has ? (uint32_t)(x / S.n) : 0u, i = has ? (uint32_t)(x % S.n) : 0u;
        if (!insert_append(S, out, ch, appended, has, has ? eps_mat[e] : 0u, i, i, make_witness(0, kWitEps, 0))) {
            add_appended(S, appended);
            return;
        }
    }
    chunk_retire(out, ch);
    add_appended(S, appended);
}

// Is `key` in the table?  Linear probing as hash_insert (tombstones are
// passed over).
__device__ __forceinline__ bool hash_contains(const unsigned long long *tab, uint64_t hmask, uint64_t key) {
    uint64_t h = mix64(key) & hmask;
    for (uint32_t p = 0; p < kMaxProbes; p++) {
        const unsigned long long v = tab[h];
        if (v == key) return true;
        if (v == kEmpty) return false;
        h = (h + 1) & hmask;
    }
    return false;
}

// A mirror plan is exact only when the seeds are their own mirror image:
// count (into ctl[kCtlMirrorMiss]) the seeds (m, i, j) whose mirror
// (mirror[m], j, i) is not in the hash set.
__global__ __launch_bounds__(256) void mirror_check_kernel(State S, PairBuf seeds, uint64_t count) {
    unsigned long long miss = 0;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < count;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t m = seeds.key[p];
        if (m == kHoleKey) continue;
        if (!hash_contains(S.hash, S.hash_mask, pair_key(S.mirror[m], seeds.j[p], seeds.i[p]))) miss++;
    }
    miss = wave_sum64(miss);
    if (lane_id() == 0 && miss) atomicAdd(&S.ctl[kCtlMirrorMiss], miss);
}

// The hash slot holding `key`, or ~0 when it is not in the table.
__device__ __forceinline__ uint64_t hash_slot(const unsigned long long *tab, uint64_t hmask, uint64_t key) {
    uint64_t h = mix64(key) & hmask;
    for (uint32_t p = 0; p < kMaxProbes; p++) {
        const unsigned long long v = tab[h];
        if (v == key) return h;
        if (v == kEmpty) return ~0ull;
        h = (h + 1) & hmask;
    }
    return ~0ull;
}

// Mirror plans: after a round's product, insert the mirror (mirror[m], j, i)
// of each of the round's first `count` new pairs (m, i, j) and append the
// ones that are new behind them, with the mirror production in the witness;
// a pair whose mirror takes no part in the rounds (mirror_ins[m] = kNone) is
// only counted (ctl[kCtlMirrorSkip]).  A re-run after an overflow covers the
// same `count` pairs: mirrors already appended are found present.
__global__ __launch_bounds__(256) void mirror_kernel(State S, PairBuf out, uint64_t count) {
    Chunk ch;
    uint64_t appended = 0, skipped = 0;
    for (uint64_t base = wave_global_id() * 64; base < count; base += waves_in_grid() * 64) {
        const uint64_t p = base + lane_id();
        uint32_t m = kHoleKey, i = 0, j = 0;
        if (p < count) {
            m = out.key[p];
            i = out.i[p];
            j = out.j[p];
        }
        const uint32_t target = m != kHoleKey ? S.mirror_ins[m] : kNone;
        if (m != kHoleKey && target == kNone) skipped++;
        const bool has = target != kNone;
        uint64_t w = 0;
        if (S.wit && has) {
            const uint64_t at = hash_slot(S.hash, S.hash_mask, pair_key(m, i, j));
            if (at != ~0ull) {
                w = S.wit[at];
                const uint32_t rule = (uint32_t)(w >> 24) & 0xFFFFFFu;
                if (rule < kWitEps) w = (w & ~(0xFFFFFFull << 24)) | ((uint64_t)(S.mirror_rule[rule] & 0xFFFFFFu) << 24);
            }
        }
        if (!insert_append(S, out, ch, appended, has, has ? target : 0u, j, i, w)) {
            add_appended(S, appended);
            return;
        }
    }
    chunk_retire(out, ch);
    add_appended(S, appended);
    skipped = wave_sum64(skipped);
    if (lane_id() == 0 && skipped) atomicAdd(&S.ctl[kCtlMirrorSkip], (unsigned long long)skipped);
}

// A sorted entry of the key sort: matrix, key vertex, partner vertex.
__device__ __forceinline__ uint64_t pack_entry(uint32_t x, uint32_t key, uint32_t partner) {
    return ((uint64_t)x << 48) | ((uint64_t)key << 24) | (uint64_t)partner;
}

// --------------------------------------------------------------- integrate

// Reset the round's counters (touched rows, planned allocation, tasks,
// moves).
__global__ void round_start_kernel(State S) {
    S.ctl[kCtlTouched] = 0;
    S.ctl[kCtlAlloc] = 0;
    S.ctl[kCtlTasks] = 0;
    S.ctl[kCtlMoves] = 0;
    S.ctl[kCtlNew] = 0;
    S.ctl[kCtlHeavy] = 0;
    S.ctl[kCtlLight] = 0;
    S.ctl[kCtlHeavyTasks] = 0;
}

// Runs of equal list index among consecutive lanes (the products emit many
// pairs of one row together): the lane's rank in its run, the run's first
// lane and, for that lane, the run's length.  kNoList marks no list.
constexpr uint64_t kNoList = ~0ull;

struct Run {
    uint32_t rank, head, len;
};

__device__ __forceinline__ Run lane_run(uint64_t idx) {
    const uint32_t lane = lane_id();
    const uint64_t prev = shfl64(idx, lane ? lane - 1 : 0);
    const uint64_t heads = __ballot(lane == 0 || prev != idx);
    const uint64_t upto = lane == 63 ? ~0ull : (2ull << lane) - 1;  // lanes <= this one
    Run r;
    r.head = 63u - (uint32_t)__builtin_clzll(heads & upto);
    r.rank = lane - r.head;
    const uint64_t after = heads & ~upto;
    r.len = (after ? (uint32_t)__builtin_ctzll(after) : 64u) - lane;
    return r;
}

// Adds a run's pairs to its list's pending count (one atomic per run); the
// list's first pending pair records it as touched.
__device__ __forceinline__ void touch(const State &S, uint64_t idx) {
    const Run r = lane_run(idx);
    uint32_t p = 1;
    if (idx != kNoList && !r.rank) p = atomicAdd(&S.cur[idx], r.len);
    const bool first = p == 0;
    const uint64_t t = wave_reserve(&S.ctl[kCtlTouched], first);
    if (!first) return;
    if (t < S.touched_cap) S.touched[t] = idx;
    else atomicOr(&S.ctl[kCtlTouchedOver], 1ull);
}

// Per pending pair: its lists' pending counts and, when the product is
// grouped (K.start set), its key-sort buckets' counts (runs of lanes with
// one bucket take one atomic), in one pass over the pairs.
__global__ __launch_bounds__(256) void count_kernel(State S, PairBuf in, KeySort K) {
    uint64_t nin = *in.count;
    if (nin > in.cap) nin = in.cap;
    const bool keys = K.start != nullptr;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x + (threadIdx.x & ~63u); base < nin; base += stride) {
        const uint64_t x = base + lane_id();
        uint64_t row = kNoList, col = kNoList, b0 = kNoList, b1 = kNoList;
        if (x < nin) {
            const uint32_t key = in.key[x];
            if (key != kHoleKey) {
                const MatInfo mi = S.mats[key];
                const uint32_t i = in.i[x], j = in.j[x];
                if (mi.app_row != kNone) row = (uint64_t)mi.app_row * S.n + i;
                if (mi.app_col != kNone) col = (uint64_t)mi.app_col * S.n + j;
                if (keys && mi.rank0 != kNone) b0 = (uint64_t)mi.rank0 * S.n + i;
                if (keys && mi.rank1 != kNone) b1 = K.nb0 + (uint64_t)mi.rank1 * S.n + j;
            }
        }
        touch(S, row);
        touch(S, col);
        if (keys) {
            const Run r0 = lane_run(b0), r1 = lane_run(b1);
            if (b0 != kNoList && !r0.rank) atomicAdd(&K.start[b0], r0.len);
            if (b1 != kNoList && !r1.rank) atomicAdd(&K.start[b1], r1.len);
        }
    }
}

__device__ __forceinline__ uint32_t grown_cap(uint32_t need) {
    uint32_t c = 2;
    while (c < need) c <<= 1;
    return c;
}

__device__ __forceinline__ uint64_t touched_count(const State &S) {
    const uint64_t t = S.ctl[kCtlTouched];
    return t < S.touched_cap ? t : S.touched_cap;
}

// The pool entries the lists that outgrow their blocks will take.
__global__ __launch_bounds__(256) void plan_kernel(State S) {
    const uint64_t nt = touched_count(S);
    uint64_t sum = 0;
    for (uint64_t base = wave_global_id() * 64; base < nt; base += waves_in_grid() * 64) {
        const uint64_t t = base + lane_id();
        if (t < nt) {
            const uint64_t idx = S.touched[t];
            const Dir d = S.dir[idx];
            const uint64_t need = (uint64_t)d.len + S.cur[idx];
            if (need > d.cap) sum += grown_cap((uint32_t)need);
        }
    }
    sum = wave_sum64(sum);
    if (lane_id() == 0 && sum) atomicAdd(&S.ctl[kCtlAlloc], (unsigned long long)sum);
}

// One thread: does the planned allocation fit the pool?  If not the round
// halts before any list moves (the host grows the pool and resumes here).
__global__ void check_kernel(State S) {
    if (S.ctl[kCtlTouchedOver]) {
        S.ctl[kCtlHalt] = 1;  // the host reports an internal error (it sizes the array to rule this out)
    } else if (S.ctl[kCtlPoolTop] + S.ctl[kCtlAlloc] > S.pool_cap) {
        S.ctl[kCtlPoolOver] = 1;
        S.ctl[kCtlHalt] = 1;
    } else {
        S.ctl[kCtlAlloc] = 0;
    }
}

// Per touched list: new length; a list that outgrows its block gets a block
// of the next power of two (short lists are copied here, longer ones are
// queued for the wave-wide copy); the cursor is set to the old length; a
// list that was empty sets its bit in every use mask that reads it.
constexpr uint32_t kInlineCopy = 16;

__global__ __launch_bounds__(256) void move_kernel(State S) {
    if (S.ctl[kCtlHalt]) return;
    const uint64_t nt = touched_count(S);
    const uint32_t lane = lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x + (threadIdx.x & ~63u); base < nt; base += stride) {
        const uint64_t t = base + lane;
        uint64_t idx = 0;
        Dir d{}, nd{};
        uint32_t pend = 0, grow = 0;
        if (t < nt) {
            idx = S.touched[t];
            d = S.dir[idx];
            pend = S.cur[idx];
            nd = d;
            nd.len = d.len + pend;
            if (nd.len > d.cap) {
                nd.cap = grown_cap(nd.len);
                grow = nd.cap;
            }
        }
        // the wave's new blocks: one reservation of the pool for all of them
        uint32_t tot;
        const uint32_t pre = wave_excl_scan(grow, &tot);
        unsigned long long top = 0;
        if (lane == 0 && tot) top = atomicAdd(&S.ctl[kCtlPoolTop], (unsigned long long)tot);
        top = first_lane64(top);
        const bool queue = grow && d.len > kInlineCopy;
        const uint64_t mv = wave_reserve(&S.ctl[kCtlMoves], queue);
        if (t >= nt) continue;
        if (grow) {
            nd.off = top + pre;
            bool queued = false;
            if (queue && mv < S.moves_cap) {
                S.moves[3 * mv] = d.off;
                S.moves[3 * mv + 1] = nd.off;
                S.moves[3 * mv + 2] = d.len;
                queued = true;
            }
            if (!queued)
                for (uint32_t q = 0; q < d.len; q++) S.pool[nd.off + q] = S.pool[d.off + q];
        }
        S.dir[idx] = nd;
        S.cur[idx] = d.len;
        if (d.len == 0) {
            const uint32_t layout = (uint32_t)(idx / S.n), r = (uint32_t)(idx % S.n);
            for (uint32_t o = S.obs_ptr[layout]; o < S.obs_ptr[layout + 1]; o++) {
                const Obs ob = S.obs[o];
                atomicOr((unsigned long long *)&S.mask[ob.base + (uint64_t)r * ob.words + ob.bit / 64],
                         1ull << (ob.bit % 64));
            }
        }
    }
}

// The queued copies of longer lists, one wave per list.
__global__ __launch_bounds__(256) void copy_kernel(State S) {
    if (S.ctl[kCtlHalt]) return;
    uint64_t nm = S.ctl[kCtlMoves];
    if (nm > S.moves_cap) nm = S.moves_cap;
    for (uint64_t w = wave_global_id(); w < nm; w += waves_in_grid()) {
        const uint64_t from = S.moves[3 * w], to = S.moves[3 * w + 1], len = S.moves[3 * w + 2];
        for (uint64_t q = lane_id(); q < len; q += 64) S.pool[to + q] = S.pool[from + q];
    }
}

// Appends value v to list idx: a run of lanes with one list takes its
// positions with one atomic.
__device__ __forceinline__ void append(const State &S, uint64_t idx, uint32_t v) {
    const Run r = lane_run(idx);
    uint32_t p = 0;
    if (idx != kNoList && !r.rank) p = atomicAdd(&S.cur[idx], r.len);
    p = shfl32(p, r.head) + r.rank;
    if (idx == kNoList) return;
    const Dir d = S.dir[idx];
    if (p < d.cap) S.pool[d.off + p] = v;
}

// Per pending pair: its entries in its lists and, when the product is
// grouped, its sorted entries (the bucket counts hold inclusive ends:
// taking a run's length off the end places its entries and, once every
// entry is placed, leaves the bucket's first position behind).
__global__ __launch_bounds__(256) void scatter_kernel(State S, PairBuf in, KeySort K) {
    if (S.ctl[kCtlHalt]) return;
    uint64_t nin = *in.count;
    if (nin > in.cap) nin = in.cap;
    const bool keys = K.start != nullptr;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x + (threadIdx.x & ~63u); base < nin; base += stride) {
        const uint64_t x = base + lane_id();
        uint64_t row = kNoList, col = kNoList, b0 = kNoList, b1 = kNoList;
        uint32_t key = 0, i = 0, j = 0;
        if (x < nin) {
            key = in.key[x];
            if (key != kHoleKey) {
                const MatInfo mi = S.mats[key];
                i = in.i[x];
                j = in.j[x];
                if (mi.app_row != kNone) row = (uint64_t)mi.app_row * S.n + i;
                if (mi.app_col != kNone) col = (uint64_t)mi.app_col * S.n + j;
                if (keys && mi.rank0 != kNone) b0 = (uint64_t)mi.rank0 * S.n + i;
                if (keys && mi.rank1 != kNone) b1 = K.nb0 + (uint64_t)mi.rank1 * S.n + j;
            }
        }
        append(S, row, j);
        append(S, col, i);
        if (keys) {
            const Run r0 = lane_run(b0), r1 = lane_run(b1);
            uint32_t p0 = 0, p1 = 0;
            if (b0 != kNoList && !r0.rank) p0 = atomicSub(&K.start[b0], r0.len);
            if (b1 != kNoList && !r1.rank) p1 = atomicSub(&K.start[b1], r1.len);
            p0 = shfl32(p0, r0.head) - 1 - r0.rank;  // the run's slots end at the old end
            p1 = shfl32(p1, r1.head) - 1 - r1.rank;
            if (b0 != kNoList && p0 < K.entry_cap) K.entry[p0] = pack_entry(key, i, j);
            if (b1 != kNoList && p1 < K.entry_cap) K.entry[p1] = pack_entry(key, j, i);
        }
    }
}

__global__ __launch_bounds__(256) void unmark_kernel(State S) {
    if (S.ctl[kCtlHalt]) return;
    const uint64_t nt = touched_count(S);
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < nt; t += (uint64_t)gridDim.x * blockDim.x)
        S.cur[S.touched[t]] = 0;
}

// ------------------------------------------------------------------ product

// first read of list `cell` (layout * n + vertex) in this round?
__device__ __forceinline__ bool first_read(const KeySort &K, uint64_t cell) {
    const uint32_t m = 1u << (cell & 31);
    return !(atomicOr(&K.touch[cell >> 5], m) & m);
}

// One lane's pair (x, pi, pj) against the partner lists of its uses in
// parts [p_lo, p_hi): the lane walks the set bits of its use masks (part 0
// at its column pj, part 1 at its row pi), one use per step, skipping the
// uses set in `skip` (when given; up to kSkipWords words); per step the
// wave expands the 64 lanes' partner lists together, each product a
// candidate inserted into the hash set.  Every lane calls this together.
// false: an overflow (the round is re-run).
constexpr uint32_t kSkipWords = 8;

__device__ __forceinline__ bool expand_uses(const State &S, const PairBuf &out, Chunk &ch, uint64_t &appended,
                                            uint64_t &products, bool valid, uint32_t x, uint32_t pi, uint32_t pj,
                                            uint32_t p_lo, uint32_t p_hi, const KeySort *acct, uint64_t &bytes,
                                            const uint64_t *skip = nullptr) {
    const uint32_t lane = lane_id();
    bool more = valid;
    MatInfo mi{};
    if (more) mi = S.mats[x];
    uint32_t part = p_lo, w = 0;
    uint64_t bits = 0;
    while (__any(more)) {
        // this lane's next use: head c, partner layout, fixed index of the
        // candidates and the partner vertex k
        uint32_t c = 0, lay = kNone, own = kNone, fixed = 0, k = 0, col = 0, rule = 0;
        if (more) {
            while (!bits) {
                const uint32_t W = part == 0 ? mi.w0 : mi.w1;
                if (part < p_hi && w < W) {
                    bits = part == 0 ? S.mask[mi.mask0 + (uint64_t)pj * mi.w0 + w]
                                     : S.mask[mi.mask1 + (uint64_t)pi * mi.w1 + w];
                    if (skip && w < kSkipWords) bits &= ~skip[w];
                    w++;
                } else if (part + 1 < p_hi) {
                    part++;
                    w = 0;
                } else {
                    more = false;
                    break;
                }
            }
            if (bits) {
                const uint32_t q = (w - 1) * 64 + (uint32_t)__builtin_ctzll(bits);
                bits &= bits - 1;
                const Use u = S.uses[(part == 0 ? mi.use0 : mi.use1) + q];
                c = u.c;
                lay = u.layout;
                own = u.own;
                rule = u.rule;
                // part 0: pair (i, k) of a meets row k of b -> (c, i, j')
                // part 1: pair (k, j) of b meets column k of a -> (c, i', j)
                fixed = part == 0 ? pi : pj;
                k = part == 0 ? pj : pi;
                col = part;
            }
        }
        uint64_t off = 0;
        uint32_t len = 0;
        if (lay != kNone) {
            const Dir d = S.dir[(uint64_t)lay * S.n + k];
            off = d.off;
            len = d.len;
            if (acct) {
                if (first_read(*acct, (uint64_t)lay * S.n + k)) bytes += 4ull * d.len;
                if (own != kNone && first_read(*acct, (uint64_t)own * S.n + fixed))
                    bytes += 4ull * S.dir[(uint64_t)own * S.n + fixed].len;
            }
        }
        uint32_t total;
        const uint32_t pre = wave_excl_scan(len, &total);
        products += total;
        for (uint32_t r = 0; r < total; r += 64) {
            const uint32_t tt = r + lane;
            uint32_t src = 0;  // last lane whose first product is <= tt
#pragma unroll
            for (uint32_t step = 32; step; step >>= 1)
                if (shfl32(pre, src + step) <= tt) src += step;
            const uint64_t soff = shfl64(off, src);
            const uint32_t spre = shfl32(pre, src), sc = shfl32(c, src), sfix = shfl32(fixed, src),
                           scol = shfl32(col, src);
            const bool has = tt < total;
            uint32_t ci = 0, cj = 0;
            if (has) {
                const uint32_t v = S.pool[soff + (tt - spre)];
                ci = scol ? v : sfix;
                cj = scol ? sfix : v;
            }
            // the witness: this production, midpoint k (the source lane's partner vertex)
            uint64_t w = 0;
            if (S.wit) w = make_witness(S.round, shfl32(rule, src), shfl32(k, src));
            if (!insert_append(S, out, ch, appended, has, sc, ci, cj, w)) return false;
        }
    }
    return true;
}

// Persistent waves; a task is 64 consecutive entries of the new-pair buffer
// `in`, one per lane, expanded against the uses of both parts.
__global__ __launch_bounds__(256) void product_kernel(State S, PairBuf in, PairBuf out) {
    const uint32_t lane = lane_id();
    uint64_t nin = *in.count;
    if (nin > in.cap) nin = in.cap;
    const uint64_t ntask = (nin + 63) / 64;
    Chunk ch;
    uint64_t appended = 0, products = 0;
    while (true) {
        unsigned long long t = 0;
        if (lane == 0) t = atomicAdd(&S.ctl[kCtlTasks], 1ull);
        t = first_lane64(t);
        if (t >= ntask) break;
        if (first_lane64(load_relaxed(&S.ctl[kCtlHalt]))) break;
        const uint64_t e = t * 64 + lane;
        uint32_t x = kHoleKey, pi = 0, pj = 0;
        if (e < nin) {
            x = in.key[e];
            pi = in.i[e];
            pj = in.j[e];
        }
        uint64_t unused = 0;
        if (!expand_uses(S, out, ch, appended, products, x != kHoleKey, x, pi, pj, 0, 2, nullptr, unused)) break;
    }
    chunk_retire(out, ch);
    add_appended(S, appended);
    if (lane == 0 && products) atomicAdd(&S.ctl[kCtlProducts], (unsigned long long)products);
}

// ----------------------------------------------------------- key-order sort


// Inclusive scan of one u32 array, three phases (block sums, their scan,
// apply).
constexpr uint32_t kScanThreads = 256, kScanItems = 16, kScanTile = kScanThreads * kScanItems;

__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const uint32_t *a, uint64_t n, uint32_t *bsum) {
    __shared__ uint32_t red[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
    for (uint32_t q = 0; q < kScanItems; q++) {
        const uint64_t x = base + q * kScanThreads + threadIdx.x;
        if (x < n) s += a[x];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t d = kScanThreads / 2; d; d >>= 1) {
        if (threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void scan_blocks_kernel(uint32_t *bsum, uint64_t nblk) {
    __shared__ uint32_t part[1024];
    __shared__ uint32_t carry;
    const uint32_t t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (uint64_t base = 0; base < nblk; base += 1024) {
        const uint32_t v = base + t < nblk ? bsum[base + t] : 0;
        part[t] = v;
        __syncthreads();
        for (uint32_t d = 1; d < 1024; d <<= 1) {
            const uint32_t u = t >= d ? part[t - d] : 0;
            __syncthreads();
            part[t] += u;
            __syncthreads();
        }
        if (base + t < nblk) bsum[base + t] = carry + part[t] - v;
        __syncthreads();
        if (t == 1023) carry += part[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(uint32_t *a, uint64_t n, const uint32_t *bsum) {
    __shared__ uint32_t tile[kScanTile];
    __shared__ uint32_t tsum[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    for (uint32_t q = 0; q < kScanItems; q++) {
        const uint64_t x = base + q * kScanThreads + threadIdx.x;
        tile[q * kScanThreads + threadIdx.x] = x < n ? a[x] : 0;
    }
    __syncthreads();
    uint32_t *mine = tile + threadIdx.x * kScanItems;
    uint32_t s = 0;
    for (uint32_t q = 0; q < kScanItems; q++) {
        s += mine[q];
        mine[q] = s;
    }
    tsum[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t d = 1; d < kScanThreads; d <<= 1) {
        const uint32_t u = threadIdx.x >= d ? tsum[threadIdx.x - d] : 0;
        __syncthreads();
        tsum[threadIdx.x] += u;
        __syncthreads();
    }
    const uint32_t off = bsum[blockIdx.x] + tsum[threadIdx.x] - s;
    for (uint32_t q = 0; q < kScanItems; q++) mine[q] += off;
    __syncthreads();
    for (uint32_t q = 0; q < kScanItems; q++) {
        const uint64_t x = base + q * kScanThreads + threadIdx.x;
        if (x < n) a[x] = tile[q * kScanThreads + threadIdx.x];
    }
}

// Products of every sorted entry (the lengths of the partner lists its use
// masks select), summed per bucket.
// The entries are in bucket order, so a wave's lanes of one bucket are
// consecutive: their products are summed over the wave first (a scan over
// runs of equal bucket) and the run's last lane adds the sum.
__global__ __launch_bounds__(256) void classify_kernel(State S, KeySort K) {
    uint64_t total = K.start[K.nb];
    if (total > K.entry_cap) total = K.entry_cap;
    const uint64_t total0 = K.start[K.nb0];
    const uint32_t lane = lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x + (threadIdx.x & ~63u); base < total; base += stride) {
        const uint64_t e = base + lane;
        uint64_t b = ~0ull, work = 0;
        if (e < total) {
            const uint64_t v = K.entry[e];
            const uint32_t x = (uint32_t)(v >> 48), key = (uint32_t)(v >> 24) & 0xFFFFFFu, k = (uint32_t)v & 0xFFFFFFu;
            const uint32_t order = e >= total0 ? 1u : 0u;
            const MatInfo mi = S.mats[x];
            const uint32_t W = order ? mi.w1 : mi.w0, first = order ? mi.use1 : mi.use0;
            const uint64_t mbase = order ? mi.mask1 : mi.mask0;
            for (uint32_t w = 0; w < W; w++) {
                uint64_t bits = S.mask[mbase + (uint64_t)k * W + w];
                while (bits) {
                    const uint32_t q = w * 64 + (uint32_t)__builtin_ctzll(bits);
                    bits &= bits - 1;
                    work += S.dir[(uint64_t)S.uses[first + q].layout * S.n + k].len;
                }
            }
            K.ework[e] = work < 0x7FFFFFFFull ? (uint32_t)work : 0x7FFFFFFFu;
            b = order ? K.nb0 + (uint64_t)mi.rank1 * S.n + key : (uint64_t)mi.rank0 * S.n + key;
        }
        uint64_t sum = work;
#pragma unroll
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint64_t ob = shfl64(b, lane >= d ? lane - d : lane);
            const uint64_t os = shfl64(sum, lane >= d ? lane - d : lane);
            if (lane >= d && ob == b) sum += os;
        }
        const uint64_t nb = shfl64(b, lane < 63 ? lane + 1 : lane);
        if (b != ~0ull && sum && (lane == 63 || nb != b)) atomicAdd(&K.work[b], (unsigned long long)sum);
    }
}

// Items: the runs of a heavy bucket's entries that do not cross a multiple
// of kHeavyRun in the sorted order (at most kHeavyRun entries each): the
// bucket's first entry and every multiple of kHeavyRun inside it.  The
// entries of the other buckets are listed for the light kernel.  One lane
// per bucket; a wave reserves the slots of all its items (entries) at once.
__global__ __launch_bounds__(256) void heavy_items_kernel(State S, KeySort K) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x + (threadIdx.x & ~63u); base < K.nb; base += stride) {
        const uint64_t b = base + lane_id();
        uint32_t s0 = 0, s1 = 0, items = 0, light = 0;
        if (b < K.nb) {
            s0 = K.start[b];
            s1 = K.start[b + 1];
            if (s1 > K.entry_cap) s1 = (uint32_t)K.entry_cap;
            if (s1 > s0) {
                if (K.work[b] >= K.threshold) items = (s1 - 1) / kHeavyRun - s0 / kHeavyRun + 1;
                else light = s1 - s0;
            }
        }
        uint32_t tot;
        const uint32_t pre = wave_excl_scan(items, &tot);
        unsigned long long h0 = 0;
        if (lane_id() == 0 && tot) h0 = atomicAdd(&S.ctl[kCtlHeavy], (unsigned long long)tot);
        h0 = first_lane64(h0);
        for (uint32_t q = 0; q < items; q++) {
            const uint64_t h = h0 + pre + q;
            const uint32_t e = q == 0 ? s0 : (s0 / kHeavyRun + q) * kHeavyRun;
            if (h < K.heavy_cap) K.heavy[h] = e;
        }
        uint32_t ltot;
        const uint32_t lpre = wave_excl_scan(light, &ltot);
        unsigned long long l0 = 0;
        if (lane_id() == 0 && ltot) l0 = atomicAdd(&S.ctl[kCtlLight], (unsigned long long)ltot);
        l0 = first_lane64(l0);
        for (uint32_t q = 0; q < light; q++)
            if (l0 + lpre + q < K.light_cap) K.light[l0 + lpre + q] = s0 + q;
    }
}

// ---------------------------------------------------------- grouped product

// Heavy items (never launched with items when witnesses are kept: a
// candidate of the bit set has lost its midpoint), one workgroup each (taken from a counter): a run of at most
// kHeavyRun entries of one bucket, thread t holding entry t.  For every use
// q selected by some entry of the item, the partner lists of the entries
// selecting it are ORed into an LDS bit set over the n columns (the lists'
// lengths prefix-summed over the workgroup, 256 consecutive products per
// pass); the pairs the head c already holds at this key are cleared from it
// (c's list in the same orientation, when c has one); the remaining bits
// are the item's candidates for c, each inserted into the hash set once.
// The bit set is left zero for the next use.
constexpr uint32_t kMaxUseWords = 8;  // uses selected through an LDS OR of the masks (512)
constexpr uint32_t kUnroll = 8;       // passes of products whose loads are issued together
constexpr uint32_t kTouchCap = 512;   // words listed as set; past that the whole bit set is scanned

// The first use at or after `from` that some entry of the item selects (its
// bit in the OR of the entries' masks; every use when the masks were not
// gathered), else nuse.
__device__ __forceinline__ uint32_t next_use(const uint64_t *um, bool gathered, uint32_t nuse, uint32_t from) {
    while (from < nuse) {
        const uint32_t w = from / 64;
        const uint64_t bits = (gathered ? um[w] : ~0ull) & (~0ull << (from % 64));
        if (bits) {
            const uint32_t q = w * 64 + (uint32_t)__builtin_ctzll(bits);
            return q < nuse ? q : nuse;
        }
        from = (w + 1) * 64;
    }
    return nuse;
}

// A use of a heavy item as one thread sees it: the production, the
// partner list at its entry's partner vertex (empty when its entry does
// not select the use) and the head's own list at the item's key.
struct UseLoad {
    Use u;
    uint64_t off;
    uint32_t len;
    Dir own;
};

template <bool kAcct>
__device__ __forceinline__ UseLoad load_use(const State &S, const KeySort &K, uint32_t q, uint32_t nuse,
                                            uint32_t first, bool mine, uint32_t k, uint32_t key, uint64_t m0,
                                            uint64_t m1, uint64_t mbase, uint32_t W, uint64_t &bytes) {
    UseLoad L{};
    L.u.own = kNone;
    if (q >= nuse) return L;
    L.u = S.uses[first + q];
    bool sel = false;
    if (mine) {
        const uint64_t m = q < 64 ? m0 : q < 128 ? m1 : S.mask[mbase + (uint64_t)k * W + q / 64];
        sel = (m >> (q % 64)) & 1;
    }
    if (sel) {
        const Dir d = S.dir[(uint64_t)L.u.layout * S.n + k];
        L.off = d.off;
        L.len = d.len;
        if (kAcct && first_read(K, (uint64_t)L.u.layout * S.n + k)) bytes += 4ull * d.len;
    }
    if (L.u.own != kNone) L.own = S.dir[(uint64_t)L.u.own * S.n + key];
    return L;
}

// Product tt of a use -> the entry (thread) whose list holds it and the
// position in that list.  pre: the wave-local exclusive prefix sums of the
// entries' list lengths; o1..o3: the first product of waves 1..3.  The wave
// is the number of wave offsets at or below tt (a wave with no products is
// skipped, as its offset equals the next one's); within it, the last lane
// whose first product is at or below tt (a lane with an empty list shares
// its prefix with a later lane, which wins).
__device__ __forceinline__ uint32_t locate(const uint32_t *pre, uint32_t o1, uint32_t o2, uint32_t o3, uint32_t tt,
                                           uint32_t *rel) {
    const uint32_t w = (uint32_t)(tt >= o1) + (uint32_t)(tt >= o2) + (uint32_t)(tt >= o3);
    const uint32_t lo = w == 0 ? 0u : w == 1 ? o1 : w == 2 ? o2 : o3;
    const uint32_t x = tt - lo;
    uint32_t src = w * 64;
#pragma unroll
    for (uint32_t step = 32; step; step >>= 1)
        if (pre[src + step] <= x) src += step;
    *rel = x - pre[src];
    return src;
}

// kAcct: the accounting variant (algorithmic bytes into K.acct), launched
// only by solves that ask for it.
template <bool kAcct>
__global__ __launch_bounds__(kHeavyThreads) void heavy_kernel(State S, KeySort K, PairBuf out) {
    extern __shared__ uint32_t acc[];
    __shared__ uint64_t um[kMaxUseWords];
    // per use, alternating between two buffers so that one barrier per use
    // suffices: a use's buffers are written again two uses later, after
    // every thread has passed the next use's barrier.  List offsets are
    // even (blocks of at least two entries from an even pool top) and held
    // halved in 32 bits (the host keeps the pool below 2^33 entries for the
    // heavy items); with the 512-word list this keeps the static LDS near
    // 6 KiB, so five workgroups fit a CU at 200,000 vertices.
    __shared__ uint32_t s_off[2][kHeavyThreads];
    __shared__ uint32_t s_pre[2][kHeavyThreads];
    __shared__ uint32_t wsum[2][kHeavyThreads / 64];
    __shared__ uint32_t sh_ntouch[2];
    __shared__ uint32_t s_touch[kTouchCap];
    __shared__ uint64_t ubig[kMaxUseWords];  // uses whose products go through the bit set
    __shared__ unsigned long long sh_item;
    __shared__ uint32_t sh_fail;
    constexpr uint32_t kWaves = kHeavyThreads / 64;
    const uint32_t t = threadIdx.x, lane = lane_id(), wave = t / 64;
    const uint32_t nw = (S.n + 31) / 32;
    uint64_t nheavy = S.ctl[kCtlHeavy];
    if (nheavy > K.heavy_cap) nheavy = K.heavy_cap;
    Chunk ch;
    uint64_t appended = 0, products = 0, cands = 0, bytes = 0;
    uint64_t wprod = 0;  // this wave's products of small uses
    for (uint32_t w = t; w < nw; w += kHeavyThreads) acc[w] = 0;
    if (t == 0) {
        sh_fail = 0;
        sh_ntouch[0] = sh_ntouch[1] = 0;
    }
    // each wave emits the candidates of words [wave * per, (wave + 1) * per)
    const uint32_t per = ((nw + kWaves - 1) / kWaves + 63) / 64 * 64;
    uint32_t par = 0;
    while (true) {
        __syncthreads();
        if (t == 0) {
            // an overflow here or elsewhere ends the launch at an item boundary
            unsigned long long it = atomicAdd(&S.ctl[kCtlHeavyTasks], 1ull);
            if (sh_fail || load_relaxed(&S.ctl[kCtlHalt])) it = nheavy;
            sh_item = it;
        }
        __syncthreads();
        const uint64_t h = sh_item;
        if (h >= nheavy) break;
        // the item: entries [e0, e1) of one bucket
        const uint32_t e0 = K.heavy[h];
        const uint64_t head = K.entry[e0];
        const uint32_t x = (uint32_t)(head >> 48), key = (uint32_t)(head >> 24) & 0xFFFFFFu;
        const uint32_t order = e0 >= K.start[K.nb0] ? 1u : 0u;
        const MatInfo mi = S.mats[x];
        const uint64_t b = order ? K.nb0 + (uint64_t)mi.rank1 * S.n + key : (uint64_t)mi.rank0 * S.n + key;
        // the item ends with its bucket or at the next multiple of kHeavyRun
        const uint32_t bend = K.start[b + 1], run_end = (e0 / kHeavyRun + 1) * kHeavyRun;
        const uint32_t cnt = (bend < run_end ? bend : run_end) - e0;
        if (t < kMaxUseWords) um[t] = 0;
        __syncthreads();
        if (kAcct && t == 0) bytes += 8ull * cnt;
        const uint32_t W = order ? mi.w1 : mi.w0, first = order ? mi.use1 : mi.use0,
                       nuse = order ? mi.nuse1 : mi.nuse0;
        const uint64_t mbase = order ? mi.mask1 : mi.mask0;
        const bool gathered = W <= kMaxUseWords;
        const bool mine = t < cnt;
        const uint32_t k = mine ? (uint32_t)K.entry[e0 + t] & 0xFFFFFFu : 0u;
        // this entry's first two mask words stay in registers
        uint64_t m0 = 0, m1 = 0;
        if (mine)
            for (uint32_t w = 0; w < W; w++) {
                const uint64_t m = S.mask[mbase + (uint64_t)k * W + w];
                if (w == 0) m0 = m;
                if (w == 1) m1 = m;
                if (gathered && m) atomicOr((unsigned long long *)&um[w], (unsigned long long)m);
            }
        __syncthreads();
        // Each selected use's products over the item (its entries' list
        // lengths summed in LDS, in the word list's space, free between
        // items).  A use with at most K.direct of them skips the bit set:
        // each wave inserts its own entries' products into the hash set, with
        // no barrier; the others go through the bit set below.
        if (gathered) {
            uint32_t *tot = s_touch;
            for (uint32_t q2 = t; q2 < nuse; q2 += kHeavyThreads) tot[q2] = 0;
            if (t < kMaxUseWords) ubig[t] = 0;
            __syncthreads();
            if (mine)
                for (uint32_t w = 0; w < W; w++) {
                    uint64_t bits = w == 0 ? m0 : w == 1 ? m1 : S.mask[mbase + (uint64_t)k * W + w];
                    while (bits) {
                        const uint32_t q2 = w * 64 + (uint32_t)__builtin_ctzll(bits);
                        bits &= bits - 1;
                        const uint32_t len = S.dir[(uint64_t)S.uses[first + q2].layout * S.n + k].len;
                        if (len) atomicAdd(&tot[q2], len);
                    }
                }
            __syncthreads();
            for (uint32_t q2 = t; q2 < nuse; q2 += kHeavyThreads)
                if (tot[q2] > K.direct) atomicOr((unsigned long long *)&ubig[q2 / 64], 1ull << (q2 % 64));
            __syncthreads();
            // each lane walks its own entry's small uses, the wave expanding
            // the 64 lanes' lists together (lanes at different uses at once)
            const bool wok = expand_uses(S, out, ch, appended, wprod, mine, x, order ? k : key, order ? key : k,
                                         order, order + 1, kAcct ? &K : nullptr, bytes, ubig);
            if (!wok && lane == 0) atomicOr(&sh_fail, 1u);
        }
        // the other uses, in order, each loaded one use ahead
        const uint64_t *sel_uses = gathered ? ubig : um;
        uint32_t q = next_use(sel_uses, gathered, nuse, 0);
        UseLoad cur = load_use<kAcct>(S, K, q, nuse, first, mine, k, key, m0, m1, mbase, W, bytes);
        while (q < nuse) {
            const uint32_t qn = next_use(sel_uses, gathered, nuse, q + 1);
            const UseLoad nxt = load_use<kAcct>(S, K, qn, nuse, first, mine, k, key, m0, m1, mbase, W, bytes);
            const Use u = cur.u;
            uint32_t wt;
            const uint32_t wpre = wave_excl_scan(cur.len, &wt);
            s_pre[par][t] = wpre;
            s_off[par][t] = (uint32_t)(cur.off >> 1);
            if (lane == 0) wsum[par][wave] = wt;
            __syncthreads();  // the use's lists are in LDS; the previous use is done
            if (t == 0) sh_ntouch[par ^ 1] = 0;  // counted into by the next use
            const uint32_t *pre = s_pre[par];
            const uint32_t *offs = s_off[par];
            const uint32_t o1 = wsum[par][0], o2 = o1 + wsum[par][1], o3 = o2 + wsum[par][2];
            const uint32_t total = o3 + wsum[par][3];
            products += total;
            if (total <= K.direct) {
                // few products: each one goes to the hash set as it is
                cands += total;
                for (uint32_t r = 0; r < total; r += kHeavyThreads) {
                    const uint32_t tt = r + t;
                    uint32_t v = 0;
                    if (tt < total) {
                        uint32_t rel;
                        const uint32_t src = locate(pre, o1, o2, o3, tt, &rel);
                        v = S.pool[2 * (uint64_t)offs[src] + rel];
                    }
                    if (!insert_append(S, out, ch, appended, tt < total, u.c, order ? v : key, order ? key : v, 0)) {
                        if (lane == 0) atomicOr(&sh_fail, 1u);
                        break;
                    }
                }
                par ^= 1;
                q = qn;
                cur = nxt;
                continue;
            }
            for (uint32_t r = 0; r < total; r += kHeavyThreads * kUnroll) {
                uint32_t v[kUnroll];
#pragma unroll
                for (uint32_t uu = 0; uu < kUnroll; uu++) {
                    const uint32_t tt = r + uu * kHeavyThreads + t;
                    v[uu] = 0xFFFFFFFFu;
                    if (tt < total) {
                        uint32_t rel;
                        const uint32_t src = locate(pre, o1, o2, o3, tt, &rel);
                        v[uu] = S.pool[2 * (uint64_t)offs[src] + rel];
                    }
                }
                // the first product into a word lists it (one thread sees it zero)
#pragma unroll
                for (uint32_t uu = 0; uu < kUnroll; uu++)
                    if (v[uu] != 0xFFFFFFFFu && !atomicOr(&acc[v[uu] >> 5], 1u << (v[uu] & 31))) {
                        const uint32_t slot = atomicAdd(&sh_ntouch[par], 1u);
                        if (slot < kTouchCap) s_touch[slot] = v[uu] >> 5;
                    }
            }
            // the head's pairs at the key count as read whether or not they are cleared
            if (kAcct && t == 0 && u.own != kNone && first_read(K, (uint64_t)u.own * S.n + key))
                bytes += 4ull * cur.own.len;
            if (u.own != kNone && (uint64_t)cur.own.len <= (uint64_t)K.row_factor * total) {
                __syncthreads();  // every product is in the bit set
                for (uint32_t p = t; p < cur.own.len; p += kHeavyThreads) {
                    const uint32_t v = S.pool[cur.own.off + p];
                    atomicAnd(&acc[v >> 5], ~(1u << (v & 31)));
                }
            }
            __syncthreads();  // the bit set holds the use's candidates
            // the listed words, else every word; each wave a quarter.  The
            // words are zeroed as they are read; the next use writes the bit
            // set only after its barrier.
            const uint32_t ntouch = sh_ntouch[par];
            const bool listed = ntouch <= kTouchCap;
            const uint32_t span = listed ? ntouch : nw;
            const uint32_t per_w = listed ? ((ntouch + kWaves - 1) / kWaves + 63) / 64 * 64 : per;
            const uint32_t w_end = (wave + 1) * per_w < span ? (wave + 1) * per_w : span;
            bool ok = true;
            for (uint32_t base = wave * per_w; base < w_end; base += 64) {
                uint32_t wi = base + lane;
                uint32_t word = 0;
                if (wi < w_end) {
                    if (listed) wi = s_touch[wi];
                    word = acc[wi];
                    acc[wi] = 0;
                }
                if (!ok) continue;
                uint32_t ctot;
                const uint32_t cpre = wave_excl_scan((uint32_t)__popc(word), &ctot);
                cands += ctot;
                for (uint32_t r = 0; r < ctot; r += 64) {
                    const uint32_t tt = r + lane;
                    uint32_t src = 0;
#pragma unroll
                    for (uint32_t step = 32; step; step >>= 1)
                        if (shfl32(cpre, src + step) <= tt) src += step;
                    const uint32_t sword = shfl32(word, src);
                    uint32_t rank = tt - shfl32(cpre, src), bit = 0;
#pragma unroll
                    for (uint32_t width = 16; width; width >>= 1) {
                        const uint32_t c2 = (uint32_t)__popc((sword >> bit) & ((1u << width) - 1));
                        if (rank >= c2) {
                            rank -= c2;
                            bit += width;
                        }
                    }
                    const bool has = tt < ctot;
                    const uint32_t v = shfl32(wi, src) * 32 + bit;
                    if (!insert_append(S, out, ch, appended, has, u.c, order ? v : key, order ? key : v, 0)) {
                        ok = false;
                        break;
                    }
                }
            }
            if (!ok && lane == 0) atomicOr(&sh_fail, 1u);
            par ^= 1;
            q = qn;
            cur = nxt;
        }
    }
    chunk_retire(out, ch);
    add_appended(S, appended);
    if (t == 0 && products) {
        atomicAdd(&S.ctl[kCtlProducts], (unsigned long long)products);
        atomicAdd(&S.ctl[kCtlHeavyProducts], (unsigned long long)products);
    }
    if (lane == 0 && wprod) {
        atomicAdd(&S.ctl[kCtlProducts], (unsigned long long)wprod);
        atomicAdd(&S.ctl[kCtlHeavyProducts], (unsigned long long)wprod);
    }
    cands += wprod;
    if (lane == 0 && cands) atomicAdd(&S.ctl[kCtlHeavyCand], (unsigned long long)cands);
    if (kAcct) {
        if (lane == 0) bytes += 16ull * appended;
        if (bytes) atomicAdd(K.acct, (unsigned long long)bytes);
    }
}

// Light buckets: 64 listed entries per task, a lane per entry, expanded
// against the uses of its own part.
// A wave claims kLightClaim tasks at a time (one counter serves them all).
constexpr uint32_t kLightClaim = 16;
template <bool kAcct>
__global__ __launch_bounds__(256) void light_kernel(State S, KeySort K, PairBuf out) {
    const uint32_t lane = lane_id();
    uint64_t total = S.ctl[kCtlLight];
    if (total > K.light_cap) total = K.light_cap;
    const uint64_t total0 = K.start[K.nb0];
    const uint64_t ntask = (total + 63) / 64;
    Chunk ch;
    uint64_t appended = 0, products = 0, bytes = 0;
    const KeySort *acct = kAcct ? &K : nullptr;
    uint64_t t = 0, t_end = 0;  // this wave's claimed tasks
    for (;; t++) {
        if (t == t_end) {
            unsigned long long c = 0;
            if (lane == 0) c = atomicAdd(&S.ctl[kCtlTasks], (unsigned long long)kLightClaim);
            t = first_lane64(c);
            if (t >= ntask) break;
            t_end = t + kLightClaim < ntask ? t + kLightClaim : ntask;
        }
        if (first_lane64(load_relaxed(&S.ctl[kCtlHalt]))) break;
        const uint64_t q = t * 64 + lane;
        const bool valid = q < total;
        uint32_t x = 0, pi = 0, pj = 0, order = 0;
        if (valid) {
            const uint32_t e = K.light[q];
            const uint64_t v = K.entry[e];
            x = (uint32_t)(v >> 48);
            const uint32_t key = (uint32_t)(v >> 24) & 0xFFFFFFu, k = (uint32_t)v & 0xFFFFFFu;
            order = e >= total0 ? 1u : 0u;
            pi = order ? k : key;
            pj = order ? key : k;
        }
        if (acct && valid) bytes += 8;
        if (!expand_uses(S, out, ch, appended, products, valid, x, pi, pj, order, order + 1, acct, bytes)) break;
    }
    chunk_retire(out, ch);
    add_appended(S, appended);
    if (lane == 0 && products) atomicAdd(&S.ctl[kCtlProducts], (unsigned long long)products);
    if (kAcct) {
        if (lane == 0) bytes += 16ull * appended;
        if (bytes) atomicAdd(K.acct_light, (unsigned long long)bytes);
    }
}

// ------------------------------------------------------------------- rehash

__global__ __launch_bounds__(256) void rehash_kernel(State S, const unsigned long long *old_tab,
                                                     const unsigned long long *old_wit, uint64_t old_slots) {
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < old_slots;
         x += (uint64_t)gridDim.x * blockDim.x) {
        const unsigned long long v = old_tab[x];
        if (v == kEmpty || v == kTomb) continue;
        uint64_t where = 0;
        const int r = hash_insert(S.hash, S.hash_mask, v, &where);
        if (r == kFull) {
            atomicOr(&S.ctl[kCtlHashFull], 1ull);
            atomicOr(&S.ctl[kCtlHalt], 1ull);
        } else if (r == kInserted && S.wit) {
            S.wit[where] = old_wit[x];
        }
    }
}

// ---------------------------------------------------------------- witnesses

// Per pair: its slot in the hash set (linear probing as inserted; every
// pair read out is in the set), its witness decoded into the grammar
// text's symbols.  A pair not found (none should be) is counted in
// *missing and gets round = CFLR_NONE.
__global__ __launch_bounds__(256) void witness_kernel(const unsigned long long *tab, uint64_t hmask,
                                                      const unsigned long long *wit, uint32_t x, const uint32_t *src,
                                                      const uint32_t *dst, uint64_t count, const uint32_t *prod_sym,
                                                      uint32_t nprod, const uint32_t *label_sym, uint32_t nlabels,
                                                      uint32_t *left, uint32_t *right, uint32_t *mid, uint32_t *round,
                                                      unsigned long long *missing) {
    constexpr uint32_t kNoSym = 0xFFFFFFFFu;
    for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < count;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t key = pair_key(x, src[p], dst[p]);
        uint64_t h = mix64(key) & hmask;
        bool found = false;
        for (uint64_t probes = 0; probes <= hmask; probes++) {
            const unsigned long long v = tab[h];
            if (v == key) {
                found = true;
                break;
            }
            if (v == kEmpty) break;
            h = (h + 1) & hmask;
        }
        uint32_t l = kNoSym, r = kNoSym, md = kNoSym, rd = kNoSym;
        bool ok = found;
        if (found) {
            const uint64_t w = wit[h];
            const uint32_t code = (uint32_t)(w >> 24) & 0xFFFFFFu, low = (uint32_t)w & 0xFFFFFFu;
            rd = (uint32_t)(w >> 48);
            if (code == kWitEdge) {
                ok = low < nlabels;
                if (ok) l = label_sym[low];
            } else if (code != kWitEps) {
                ok = code < nprod;
                if (ok) {
                    l = prod_sym[2 * (uint64_t)code];
                    r = prod_sym[2 * (uint64_t)code + 1];
                    md = low;
                }
            }
        }
        if (!ok) {
            rd = kNoSym;
            atomicAdd(missing, 1ull);
        }
        left[p] = l;
        right[p] = r;
        mid[p] = md;
        round[p] = rd;
    }
}

__global__ void check_edges_kernel(const uint32_t *src, const uint32_t *dst, const uint32_t *lab, uint64_t m,
                                   uint32_t n, uint32_t n_labels, unsigned long long *bad) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x)
        if (src[e] >= n || dst[e] >= n || lab[e] >= n_labels) atomicOr(bad, 1ull);
}

__global__ void fill_u64_kernel(unsigned long long *a, uint64_t n, unsigned long long v) {
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n; x += (uint64_t)gridDim.x * blockDim.x)
        a[x] = v;
}

__global__ void fill_u32_kernel(uint32_t *a, uint64_t n, uint32_t v) {
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n; x += (uint64_t)gridDim.x * blockDim.x)
        a[x] = v;
}

// ------------------------------------------------------------------ readout

// Transposed readout (a matrix whose pairs are read from its mirror's row
// layout): cnt[j] += 1 for every entry j of every list, a wave per list.
__global__ __launch_bounds__(256) void transpose_count_kernel(const Dir *dir, const uint32_t *pool, uint32_t n,
                                                             uint32_t *cnt) {
    for (uint64_t i = wave_global_id(); i < n; i += waves_in_grid()) {
        const Dir d = dir[i];
        for (uint32_t e = lane_id(); e < d.len; e += 64) atomicAdd(&cnt[pool[d.off + e]], 1u);
    }
}

// Every entry j of list i goes to tdir[j]'s block as i (unsorted within the
// block; the row readout sorts it).
__global__ __launch_bounds__(256) void transpose_scatter_kernel(const Dir *dir, const uint32_t *pool, uint32_t n,
                                                               const Dir *tdir, uint32_t *cursor, uint32_t *tpool) {
    for (uint64_t i = wave_global_id(); i < n; i += waves_in_grid()) {
        const Dir d = dir[i];
        for (uint32_t e = lane_id(); e < d.len; e += 64) {
            const uint32_t j = pool[d.off + e];
            const uint32_t at = atomicAdd(&cursor[j], 1u);
            tpool[tdir[j].off + at] = (uint32_t)i;
        }
    }
}

__global__ __launch_bounds__(256) void layout_count_kernel(const Dir *dir, uint32_t n, unsigned long long *total) {
    uint64_t s = 0;
    for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < n; r += (uint64_t)gridDim.x * blockDim.x)
        s += dir[r].len;
    s = wave_sum64(s);
    if (lane_id() == 0 && s) atomicAdd(total, (unsigned long long)s);
}

// exclusive scan of the list lengths into 64-bit offsets, one workgroup
__global__ __launch_bounds__(1024) void offsets_kernel(const Dir *dir, uint32_t n, uint64_t *off) {
    __shared__ uint64_t part[1024];
    __shared__ uint64_t carry;
    const uint32_t t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < n; base += 1024) {
        const uint64_t v = base + t < n ? dir[base + t].len : 0;
        part[t] = v;
        __syncthreads();
        for (uint32_t d = 1; d < 1024; d <<= 1) {
            const uint64_t u = t >= d ? part[t - d] : 0;
            __syncthreads();
            part[t] += u;
            __syncthreads();
        }
        if (base + t < n) off[base + t] = carry + part[t] - v;
        __syncthreads();
        if (t == 1023) carry += part[1023];
        __syncthreads();
    }
}

// Rows in (i, j) order: one workgroup per row.  A list of at most kSortMax
// entries is sorted in LDS (bitonic); a longer one is put into a bit set of
// the n columns (this workgroup's part of `bitmap`, zero between rows) and
// read back in column order.
constexpr uint32_t kSortThreads = 256, kSortMax = 2048;

__global__ __launch_bounds__(kSortThreads) void row_write_kernel(const Dir *dir, const uint32_t *pool, uint32_t n,
                                                                 const uint64_t *off, uint64_t *bitmap,
                                                                 uint32_t *src, uint32_t *dst) {
    __shared__ uint32_t v[kSortMax];
    __shared__ uint32_t cnt[kSortThreads];
    const uint32_t t = threadIdx.x;
    const uint64_t nw = ((uint64_t)n + 63) / 64;
    uint64_t *bm = bitmap + (uint64_t)blockIdx.x * nw;
    for (uint32_t r = blockIdx.x; r < n; r += gridDim.x) {
        const Dir d = dir[r];
        const uint64_t o = off[r];
        if (d.len == 0) continue;
        if (d.len <= kSortMax) {
            uint32_t m = 2;
            while (m < d.len) m <<= 1;
            for (uint32_t q = t; q < m; q += kSortThreads) v[q] = q < d.len ? pool[d.off + q] : 0xFFFFFFFFu;
            __syncthreads();
            for (uint32_t k = 2; k <= m; k <<= 1) {
                for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
                    for (uint32_t q = t; q < m; q += kSortThreads) {
                        const uint32_t p = q ^ jj;
                        if (p > q) {
                            const bool up = (q & k) == 0;
                            const uint32_t a = v[q], b = v[p];
                            if ((a > b) == up) {
                                v[q] = b;
                                v[p] = a;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            for (uint32_t q = t; q < d.len; q += kSortThreads) {
                src[o + q] = r;
                dst[o + q] = v[q];
            }
            __syncthreads();
            continue;
        }
        for (uint32_t q = t; q < d.len; q += kSortThreads) {
            const uint32_t c = pool[d.off + q];
            atomicOr((unsigned long long *)&bm[c >> 6], 1ull << (c & 63));
        }
        __syncthreads();
        // thread t reads words [w0, w1) in order
        const uint64_t per = (nw + kSortThreads - 1) / kSortThreads;
        const uint64_t w0 = (uint64_t)t * per < nw ? (uint64_t)t * per : nw;
        const uint64_t w1 = w0 + per < nw ? w0 + per : nw;
        uint32_t c = 0;
        for (uint64_t w = w0; w < w1; w++) c += (uint32_t)__popcll(bm[w]);
        cnt[t] = c;
        __syncthreads();
        for (uint32_t dd = 1; dd < kSortThreads; dd <<= 1) {
            const uint32_t u = t >= dd ? cnt[t - dd] : 0;
            __syncthreads();
            cnt[t] += u;
            __syncthreads();
        }
        uint64_t p = o + cnt[t] - c;
        for (uint64_t w = w0; w < w1; w++) {
            uint64_t b = bm[w];
            bm[w] = 0;
            while (b) {
                src[p] = r;
                dst[p] = (uint32_t)(w * 64 + (uint64_t)__builtin_ctzll(b));
                b &= b - 1;
                p++;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ host launchers

#define SP_LAUNCH_CHECK()                      \
    do {                                       \
        hipError_t e_ = hipGetLastError();     \
        if (e_ != hipSuccess) return e_;       \
    } while (0)

static uint32_t grid_for(uint64_t items, uint32_t threads, uint32_t cap) {
    uint64_t g = (items + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

hipError_t launch_seed(const State &S, const uint32_t *src, const uint32_t *dst, const uint32_t *lab, uint64_t m,
                       const uint32_t *lm_ptr, const uint32_t *lm_mat, const uint32_t *eps_mat, uint32_t n_eps,
                       PairBuf out, hipStream_t s) {
    if (m) {
        seed_edges_kernel<<<grid_for(m, 256, kSeedBlocks), 256, 0, s>>>(S, src, dst, lab, m, lm_ptr, lm_mat, out);
        SP_LAUNCH_CHECK();
    }
    const uint64_t e = (uint64_t)n_eps * S.n;
    if (e) {
        seed_eps_kernel<<<grid_for(e, 256, kSeedBlocks), 256, 0, s>>>(S, eps_mat, n_eps, out);
        SP_LAUNCH_CHECK();
    }
    return hipSuccess;
}

hipError_t launch_mirror_check(const State &S, PairBuf seeds, uint64_t count, hipStream_t s) {
    if (!count) return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((count + 255) / 256, 4096);
    mirror_check_kernel<<<(uint32_t)blocks, 256, 0, s>>>(S, seeds, count);
    return hipGetLastError();
}

hipError_t launch_mirror(const State &S, PairBuf out, uint64_t count, uint32_t grid_waves, hipStream_t s) {
    if (!count) return hipSuccess;
    const uint64_t waves = std::min<uint64_t>(grid_waves, (count + 63) / 64);
    mirror_kernel<<<(uint32_t)((waves + 3) / 4), 256, 0, s>>>(S, out, count);
    return hipGetLastError();
}

hipError_t launch_round_start(const State &S, hipStream_t s) {
    round_start_kernel<<<1, 1, 0, s>>>(S);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_integrate(const State &S, PairBuf in, const KeySort *K, bool resume, uint32_t grid,
                            hipStream_t s) {
    KeySort none{};
    const KeySort &Kk = K ? *K : none;
    if (!resume) {
        if (K) {
            const uint64_t len = K->nb + 1;
            fill_u32_kernel<<<grid_for(len, 256, 65536), 256, 0, s>>>(K->start, len, 0);
            SP_LAUNCH_CHECK();
            fill_u64_kernel<<<grid_for(K->nb, 256, 65536), 256, 0, s>>>(K->work, K->nb, 0);
            SP_LAUNCH_CHECK();
        }
        count_kernel<<<grid, 256, 0, s>>>(S, in, Kk);
        SP_LAUNCH_CHECK();
        plan_kernel<<<grid, 256, 0, s>>>(S);
        SP_LAUNCH_CHECK();
    }
    check_kernel<<<1, 1, 0, s>>>(S);
    SP_LAUNCH_CHECK();
    move_kernel<<<grid, 256, 0, s>>>(S);
    SP_LAUNCH_CHECK();
    copy_kernel<<<grid, 256, 0, s>>>(S);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_integrate_finish(const State &S, PairBuf in, const KeySort *K, uint32_t grid, hipStream_t s) {
    KeySort none{};
    if (K) {
        const uint64_t len = K->nb + 1, nblk = key_sort_scan_blocks(K->nb);
        scan_reduce_kernel<<<(uint32_t)nblk, kScanThreads, 0, s>>>(K->start, len, K->bsum);
        SP_LAUNCH_CHECK();
        scan_blocks_kernel<<<1, 1024, 0, s>>>(K->bsum, nblk);
        SP_LAUNCH_CHECK();
        scan_apply_kernel<<<(uint32_t)nblk, kScanThreads, 0, s>>>(K->start, len, K->bsum);
        SP_LAUNCH_CHECK();
    }
    scatter_kernel<<<grid, 256, 0, s>>>(S, in, K ? *K : none);
    SP_LAUNCH_CHECK();
    unmark_kernel<<<grid, 256, 0, s>>>(S);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_product(const State &S, PairBuf in, PairBuf out, uint32_t grid_waves, hipStream_t s) {
    const uint32_t blocks = grid_waves / 4 ? grid_waves / 4 : 1;
    product_kernel<<<blocks, 256, 0, s>>>(S, in, out);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

uint64_t key_sort_scan_blocks(uint64_t nb) { return (nb + 1 + kScanTile - 1) / kScanTile; }

hipError_t launch_key_sort(const State &S, PairBuf in, const KeySort &K, hipStream_t s) {
    classify_kernel<<<grid_for(2 * in.cap, 256, 8192), 256, 0, s>>>(S, K);
    SP_LAUNCH_CHECK();
    heavy_items_kernel<<<grid_for(K.nb, 256, 8192), 256, 0, s>>>(S, K);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_heavy(const State &S, const KeySort &K, PairBuf out, uint32_t grid_waves, hipStream_t s) {
    const uint32_t blocks = grid_waves / 4 ? grid_waves / 4 : 1;
    if (K.acct)
        heavy_kernel<true><<<blocks, kHeavyThreads, (uint32_t)heavy_lds_bytes(S.n), s>>>(S, K, out);
    else
        heavy_kernel<false><<<blocks, kHeavyThreads, (uint32_t)heavy_lds_bytes(S.n), s>>>(S, K, out);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_light(const State &S, const KeySort &K, PairBuf out, uint32_t grid_waves, hipStream_t s) {
    const uint32_t blocks = grid_waves / 4 ? grid_waves / 4 : 1;
    if (K.acct_light)
        light_kernel<true><<<blocks, 256, 0, s>>>(S, K, out);
    else
        light_kernel<false><<<blocks, 256, 0, s>>>(S, K, out);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_rehash(const State &S, const unsigned long long *old_tab, const unsigned long long *old_wit,
                         uint64_t old_slots, hipStream_t s) {
    rehash_kernel<<<grid_for(old_slots, 256, 65536), 256, 0, s>>>(S, old_tab, old_wit, old_slots);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_witness(const unsigned long long *tab, uint64_t hmask, const unsigned long long *wit, uint32_t x,
                          const uint32_t *src, const uint32_t *dst, uint64_t count, const uint32_t *prod_sym,
                          uint32_t nprod, const uint32_t *label_sym, uint32_t nlabels, uint32_t *left,
                          uint32_t *right, uint32_t *mid, uint32_t *round, unsigned long long *missing,
                          hipStream_t s) {
    if (!count) return hipSuccess;
    witness_kernel<<<grid_for(count, 256, 65536), 256, 0, s>>>(tab, hmask, wit, x, src, dst, count, prod_sym, nprod,
                                                               label_sym, nlabels, left, right, mid, round, missing);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_fill_u64(unsigned long long *a, uint64_t n, unsigned long long v, hipStream_t s) {
    if (!n) return hipSuccess;
    fill_u64_kernel<<<grid_for(n, 256, 65536), 256, 0, s>>>(a, n, v);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_check_edges(const uint32_t *src, const uint32_t *dst, const uint32_t *lab, uint64_t m, uint32_t n,
                              uint32_t n_labels, unsigned long long *bad, hipStream_t s) {
    if (!m) return hipSuccess;
    check_edges_kernel<<<grid_for(m, 256, 8192), 256, 0, s>>>(src, dst, lab, m, n, n_labels, bad);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_fill_u32(uint32_t *a, uint64_t n, uint32_t v, hipStream_t s) {
    if (!n) return hipSuccess;
    fill_u32_kernel<<<grid_for(n, 256, 65536), 256, 0, s>>>(a, n, v);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_layout_count(const Dir *dir, uint32_t n, unsigned long long *total, hipStream_t s) {
    if (!n) return hipSuccess;
    layout_count_kernel<<<grid_for(n, 256, 4096), 256, 0, s>>>(dir, n, total);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_transpose_count(const Dir *dir, const uint32_t *pool, uint32_t n, uint32_t *cnt, hipStream_t s) {
    if (!n) return hipSuccess;
    transpose_count_kernel<<<grid_for(n, 4, 8192), 256, 0, s>>>(dir, pool, n, cnt);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_transpose_scatter(const Dir *dir, const uint32_t *pool, uint32_t n, const Dir *tdir,
                                    uint32_t *cursor, uint32_t *tpool, hipStream_t s) {
    if (!n) return hipSuccess;
    transpose_scatter_kernel<<<grid_for(n, 4, 8192), 256, 0, s>>>(dir, pool, n, tdir, cursor, tpool);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_layout_write(const Dir *dir, const uint32_t *pool, uint32_t n, uint64_t *off_scratch,
                               uint64_t *bitmap_scratch, uint32_t sort_grid, uint32_t *src, uint32_t *dst,
                               hipStream_t s) {
    if (!n) return hipSuccess;
    offsets_kernel<<<1, 1024, 0, s>>>(dir, n, off_scratch);
    SP_LAUNCH_CHECK();
    row_write_kernel<<<sort_grid, kSortThreads, 0, s>>>(dir, pool, n, off_scratch, bitmap_scratch, src, dst);
    SP_LAUNCH_CHECK();
    return hipSuccess;
}

}  // namespace sp
}  // namespace cflr

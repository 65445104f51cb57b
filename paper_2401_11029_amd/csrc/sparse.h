// sparse.h -- device data layout of the sparse storage engine.
//
// The dense engine (kernels.h) keeps every matrix as an n x n bit matrix,
// which cannot hold a grammar with hundreds of non-terminals on a large
// graph (644 matrices at 200,000 vertices would need terabytes).  This
// engine stores each relation by its pairs:
//
//  * adjacency lists: per matrix a row-major layout (row i lists the j of
//    its pairs (i, j)) when the matrix stands in a b slot of some production
//    or is a result, and a column-major layout (column j lists the i) when
//    it stands in an a slot (Section 3, optimisation 2 and its pruning: b
//    needs rows, a needs columns).  A list is a block of u32 entries in one
//    shared pool with a capacity; appending past it moves the list to a block
//    of twice the size, so adding the sparse new pairs of a round never
//    rebuilds a matrix (the requirement of Section 3, optimisation 3) and
//    every entry is copied O(1) times on average;
//  * membership: one open-addressing hash set over 64-bit keys
//    (matrix, i, j) for every matrix, probed linearly; inserting a candidate
//    with a compare-and-swap both masks it against the matrix and adds it,
//    and tells exactly one thread that the pair is new;
//  * use masks: for every matrix x and part (x in an a slot: part 0, in a b
//    slot: part 1), per vertex k a bit per production using x there, set
//    once the partner list that production would read at k (b's row k, or
//    a's column k) is non-empty.  A new pair of x reads the partner lists
//    of the productions whose bits are set, not of all of them: a
//    non-terminal used by 193 productions (points-to PT, FT) has a few
//    non-empty partners per vertex.  This is the block directory of an
//    indexed non-terminal (Section 3, optimisation 4), kept per vertex.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cflr {
namespace sp {

constexpr uint64_t kEmpty = ~0ull;      // free hash slot
constexpr uint64_t kTomb = ~0ull - 1;   // slot of a key taken back after an overflow
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kHoleKey = 0xFFFFFFFFu;  // unused entry of a new-pair buffer
constexpr uint32_t kMaxVertices = 1u << 24;  // vertex ids fit 24 bits of a key
constexpr uint32_t kMaxMatrices = 0xFFFFu;   // matrix ids fit 16 bits (0xFFFF reserved)
// New-pair buffer slots a wave reserves at a time; a wave leaves at most one
// partly used chunk (its unused slots become holes).
constexpr uint32_t kChunk = 256;
// Workgroups (of 4 waves) of each seeding kernel at most: the seed buffer
// needs 2 * 4 * kSeedBlocks * kChunk slots beyond the seeds themselves.
constexpr uint32_t kSeedBlocks = 2048;

// Hash key of pair (i, j) of matrix m; never equal to kEmpty or kTomb
// because m < 0xFFFF.
__host__ __device__ inline uint64_t pair_key(uint32_t m, uint32_t i, uint32_t j) {
    return ((uint64_t)m << 48) | ((uint64_t)i << 24) | (uint64_t)j;
}

// Witness of a pair (single-path semantics; kept per hash slot when a solve
// asks for it): the round that derived it (bits 48..63; seeds 0), what
// derived it (bits 24..47: the index of a binary production, kWitEdge or
// kWitEps) and its midpoint (bits 0..23; for an edge, the edge's graph
// label).
constexpr uint32_t kWitEdge = 0xFFFFFF, kWitEps = 0xFFFFFE, kWitMaxRound = 0xFFFF;
__host__ __device__ inline uint64_t make_witness(uint32_t round, uint32_t code, uint32_t mid) {
    const uint64_t r = round < kWitMaxRound ? round : kWitMaxRound;
    return (r << 48) | ((uint64_t)(code & 0xFFFFFF) << 24) | (uint64_t)(mid & 0xFFFFFF);
}

// One adjacency list: entries pool[off, off + len), room for cap.
struct Dir {
    uint64_t off;
    uint32_t len, cap;
};

// A production seen from one of its operands: the head c, the partner
// layout the product reads (part 0: b's row layout; part 1: a's column
// layout), c's own layout in the candidates' orientation (part 0: its row
// layout; part 1: its column layout; kNone when c has none) and the
// production's index among the binary productions (for witnesses).
struct Use {
    uint32_t c;
    uint32_t layout;
    uint32_t own;
    uint32_t rule;
};

// A use mask to update when a list of some layout becomes non-empty at
// vertex k: word base + k * words + bit / 64 of the mask array, bit % 64.
struct Obs {
    uint64_t base;
    uint32_t words;
    uint32_t bit;
};

struct MatInfo {
    uint32_t row_layout, col_layout;  // kNone when absent
    // the layouts the matrix's own pairs are appended to (kNone: none; a
    // mirror plan's column layout is the mirror's row layout, which only
    // the mirror's pairs fill)
    uint32_t app_row, app_col;
    uint32_t use0, nuse0;             // part 0 uses (x in an a slot) in the use table
    uint32_t use1, nuse1;             // part 1 uses (x in a b slot)
    uint32_t w0, w1;                  // mask words per vertex for each part
    uint64_t mask0, mask1;            // first word of each part's masks
    uint32_t rank0, rank1;            // index among the matrices with part 0 (part 1) uses; kNone if none
};

// The new pairs of a round in key order, for the grouped product: a pair
// (i, j) of a matrix x with part 0 uses goes to bucket rank0(x) * n + i
// (its key i, its partner j), and with part 1 uses to bucket
// nb0 + rank1(x) * n + j (key j, partner i).  Buckets are laid out in
// order, so all part 0 entries come first.  A bucket is one output row (part
// 0) or column (part 1) of every production using x: its products are the
// union of the partner lists its entries select.
struct KeySort {
    uint64_t nb0, nb;          // buckets of part 0; of both parts
    uint32_t *start;           // [nb + 1]: counts, then inclusive ends, then (after
                               // the scatter) the first entry of each bucket; [nb] = entries
    unsigned long long *work;  // [nb]: products of each bucket (the classification)
    uint32_t *ework;           // [entry_cap]: products of each sorted entry
    uint64_t *entry;           // sorted entries: x << 48 | key << 24 | partner
    uint64_t entry_cap;
    uint32_t *heavy;           // items of the buckets whose products reach `threshold`: the
                               // first entry of a run of at most kHeavyRun entries
    uint64_t heavy_cap;
    uint32_t *light;           // the entries of the other buckets, listed bucket by bucket
    uint64_t light_cap;
    uint64_t threshold;
    uint32_t direct;           // a heavy item's use with at most this many products inserts
                               // them into the hash set directly (no bit set)
    uint32_t row_factor;       // a heavy item clears the head's pairs at its key from the
                               // bit set only when that list is at most row_factor times
                               // the item's products for the head (else the hash set
                               // alone rejects them)
    uint32_t *bsum;            // scan scratch
    // traffic accounting (null unless counting): a bit per (layout,
    // vertex) list, set on its first read in a round, and the algorithmic
    // bytes of the heavy and the light kernel: 8 per sorted entry, 4 per
    // entry of every distinct partner list and output row (the head's list
    // at the key, the mask of the candidates) read in the round, 16 per
    // new pair
    uint32_t *touch;
    unsigned long long *acct;        // heavy kernel
    unsigned long long *acct_light;  // light kernel
};

// New pairs of a round: (matrix, i, j); kHoleKey marks an unused entry.
struct PairBuf {
    uint32_t *key, *i, *j;
    unsigned long long *count;  // entries taken (may exceed cap after an overflow)
    uint64_t cap;
};

// Everything a kernel of a round reads; all device pointers.
struct State {
    uint32_t n;
    uint32_t nlayouts;
    const MatInfo *mats;
    const Use *uses;
    const uint32_t *obs_ptr;  // [nlayouts + 1]
    const Obs *obs;
    Dir *dir;                 // [nlayouts * n]
    uint32_t *cur;            // [nlayouts * n]: pending count, then write cursor
    uint64_t *mask;           // use masks
    uint32_t *pool;
    uint64_t pool_cap;
    unsigned long long *hash;  // hash slots
    uint64_t hash_mask;        // slots - 1 (a power of two minus one)
    unsigned long long *wit;   // per hash slot, the witness of its pair (null: not kept)
    // mirror plan (null: none): per matrix its mirror, per binary production
    // its mirror production; after a round's product, the mirror pass
    // inserts (mirror[x], j, i) for each new pair (x, i, j)
    const uint32_t *mirror;
    const uint32_t *mirror_rule;
    // per matrix x: the mirror the pass inserts for x's new pairs, or kNone
    // when that mirror takes no part in the rounds (no uses, no lists of its
    // own, head of no kept production) and no witnesses are kept
    const uint32_t *mirror_ins;
    uint32_t round;            // the round being run (0 while seeding), for witnesses
    // bookkeeping words (kCtl* below)
    unsigned long long *ctl;
    uint64_t *touched;  // lists with pending entries: layout * n + row
    uint64_t touched_cap;
    uint64_t *moves;    // queued list copies: (from, to, length)
    uint64_t moves_cap;
};

constexpr int kCtlPoolTop = 0,   // pool entries handed out
    kCtlTouched = 1,             // lists touched by this round's new pairs
    kCtlAlloc = 2,               // pool entries the moves of this round need
    kCtlHalt = 3,                // an overflow: the rest of the round is skipped
    kCtlPoolOver = 4,            // the planned moves do not fit the pool
    kCtlBufOver = 5,             // a new-pair buffer is full
    kCtlTomb = 6,                // keys taken back after an overflow
    kCtlTasks = 7,               // product tasks taken
    kCtlMoves = 8,               // queued list copies
    kCtlHashFull = 9,            // an insert found no free slot
    kCtlNew = 10,                // new pairs appended (seeding, or a round's product)
    kCtlTouchedOver = 11,        // more touched lists than the array holds
    kCtlProducts = 12,           // boolean products (list entries read) of the products
    kCtlHeavy = 13,              // heavy buckets of the grouped product
    kCtlHeavyTasks = 14,         // heavy buckets taken
    kCtlHeavyProducts = 15,      // products of the heavy items
    kCtlHeavyCand = 16,          // candidates the heavy items sent to the hash set
    kCtlLight = 17,              // entries of the light buckets listed
    kCtlMirrorMiss = 18,         // seeds whose mirror pair is missing (mirror plans)
    kCtlMirrorSkip = 19,         // new pairs whose mirror the pass left out (mirror_ins)
    kCtlWords = 20;

// ------------------------------------------------------------------ launchers

// Seeding: every edge (u, t, v) gives (x, u, v) for every x -> t, and every
// x -> eps gives (x, i, i) for all i; new pairs go to `out`.
hipError_t launch_seed(const State &S, const uint32_t *src, const uint32_t *dst, const uint32_t *lab, uint64_t m,
                       const uint32_t *lm_ptr, const uint32_t *lm_mat, const uint32_t *eps_mat, uint32_t n_eps,
                       PairBuf out, hipStream_t s);
// Mirror plans: count into ctl[kCtlMirrorMiss] the first `count` entries
// (m, i, j) of the seed buffer whose mirror (S.mirror[m], j, i) is not in
// the hash set (holes skipped).
hipError_t launch_mirror_check(const State &S, PairBuf seeds, uint64_t count, hipStream_t s);
// Mirror plans, after a round's product: insert the mirror of each of the
// first `count` pairs of `out` and append the new ones behind them (an
// overflow halts the pass; the host grows and re-runs it over the same
// `count` pairs).
hipError_t launch_mirror(const State &S, PairBuf out, uint64_t count, uint32_t grid_waves, hipStream_t s);
// Add the new pairs `in` to the adjacency lists, in two launches: count
// (and, with K, the key sort's bucket counts in the same pass), plan, check,
// move; then, once the pool held (launch_integrate_finish), the buckets'
// scan, the appends (and the sorted entries), reset.  With resume = true
// only the steps from the capacity check on run (after the host grew an
// overflowing pool).
hipError_t launch_integrate(const State &S, PairBuf in, const KeySort *K, bool resume, uint32_t grid,
                            hipStream_t s);
hipError_t launch_integrate_finish(const State &S, PairBuf in, const KeySort *K, uint32_t grid, hipStream_t s);
// Zero the counters a round starts from (touched lists, planned
// allocation, tasks, queued copies).
hipError_t launch_round_start(const State &S, hipStream_t s);
// The round's product: every pair of `in`, for every use whose mask bit is
// set, against the partner list; candidates inserted in the hash set; new
// ones appended to `out`.
hipError_t launch_product(const State &S, PairBuf in, PairBuf out, uint32_t grid_waves, hipStream_t s);
// The grouped product: sort the pending pairs into key order, classify the
// buckets by their products, then the heavy buckets (one workgroup each, an
// LDS bit accumulator over the n columns, kHeavyThreads threads) and the
// light ones (per product, as launch_product).
constexpr uint32_t kHeavyThreads = 256;
constexpr uint32_t kHeavyRun = kHeavyThreads;  // entries of a heavy item at most

// The key sort's last steps (after launch_integrate_finish placed the
// entries): per entry its products, the heavy items and the light list.
hipError_t launch_key_sort(const State &S, PairBuf in, const KeySort &K, hipStream_t s);
hipError_t launch_heavy(const State &S, const KeySort &K, PairBuf out, uint32_t grid_waves, hipStream_t s);
hipError_t launch_light(const State &S, const KeySort &K, PairBuf out, uint32_t grid_waves, hipStream_t s);
uint64_t key_sort_scan_blocks(uint64_t nb);
// LDS bytes of a heavy workgroup's accumulator (n bits); the grouped product
// needs n small enough for it to fit.
inline uint64_t heavy_lds_bytes(uint32_t n) { return ((uint64_t)n + 31) / 32 * 4; }
constexpr uint64_t kHeavyMaxLds = 56 * 1024;  // with the kernel's static LDS (about 6 KiB), within 64 KiB
constexpr uint64_t kHeavyMaxPool = 1ull << 33;  // pool entries whose (even) offsets the heavy items hold halved in 32 bits
// Re-insert every key of `old_tab` (tombstones dropped) into S.hash (empty).
hipError_t launch_rehash(const State &S, const unsigned long long *old_tab, const unsigned long long *old_wit,
                         uint64_t old_slots, hipStream_t s);
// Witnesses of `count` pairs (x, src[p], dst[p]) read from the hash set, in
// symbols of the grammar text: prod_sym[2q], [2q + 1] = the operands of
// binary production q < nprod, label_sym[l] = the terminal of graph label
// l < nlabels.  Pairs not found, or with a witness outside these tables,
// are counted in *missing.
hipError_t launch_witness(const unsigned long long *tab, uint64_t hmask, const unsigned long long *wit, uint32_t x,
                          const uint32_t *src, const uint32_t *dst, uint64_t count, const uint32_t *prod_sym,
                          uint32_t nprod, const uint32_t *label_sym, uint32_t nlabels, uint32_t *left,
                          uint32_t *right, uint32_t *mid, uint32_t *round, unsigned long long *missing,
                          hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *a, uint64_t n, unsigned long long v, hipStream_t s);
// *bad |= 1 if some edge has src or dst >= n or label >= n_labels.
hipError_t launch_check_edges(const uint32_t *src, const uint32_t *dst, const uint32_t *lab, uint64_t m, uint32_t n,
                              uint32_t n_labels, unsigned long long *bad, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *a, uint64_t n, uint32_t v, hipStream_t s);
// Transposed readout of a row layout (the pairs of a matrix kept only as
// its mirror's rows): cnt[j] (zeroed by the caller) counts the entries j
// over all n lists; then every entry j of list i is written as i into
// tpool at tdir[j].off + (a cursor[j] slot; cursor zeroed by the caller).
// tdir (built by the host from cnt) is then a row layout of the transpose.
hipError_t launch_transpose_count(const Dir *dir, const uint32_t *pool, uint32_t n, uint32_t *cnt, hipStream_t s);
hipError_t launch_transpose_scatter(const Dir *dir, const uint32_t *pool, uint32_t n, const Dir *tdir,
                                    uint32_t *cursor, uint32_t *tpool, hipStream_t s);
// Readout of one row layout: per-row counts (sum into *total), then the
// pairs sorted by (i, j) at the exclusive offsets of the counts.
hipError_t launch_layout_count(const Dir *dir, uint32_t n, unsigned long long *total, hipStream_t s);
hipError_t launch_layout_write(const Dir *dir, const uint32_t *pool, uint32_t n, uint64_t *off_scratch,
                               uint64_t *bitmap_scratch, uint32_t sort_grid, uint32_t *src, uint32_t *dst,
                               hipStream_t s);

}  // namespace sp
}  // namespace cflr
